// gf_api.cpp -- host side of libgf: contexts, batches, PSF preparation
// (FFT plans, OTFs, work lists), the step 1-3 entry points, derivatives and
// the device-resident Levenberg-Marquardt driver.
#include <algorithm>
#include <atomic>
#include <map>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gf_internal.h"

namespace gf {
std::vector<float4> build_bn_table();
hipError_t noalloc_init(int device);
hipError_t launch_eval(hipStream_t, const gf_batch *, const float *, int, const float4 *, float *, const int *);
hipError_t launch_eval_d(hipStream_t, const gf_batch *, const double *, int, const float4 *, float *, const int *,
                         const WorkView *, CompC *cc = nullptr, bool prep = true);
hipError_t launch_eval_jac(hipStream_t, const gf_batch *, const float *, int, const float4 *, float *, int,
                           const int *);
hipError_t launch_eval_jac_d(hipStream_t, const gf_batch *, const double *, int, const float4 *, float *, int,
                             const int *, const WorkView *, CompC *cc = nullptr, bool prep = true);
hipError_t launch_adjoint_contract(hipStream_t, const gf_batch *, const float *, int, const float4 *, const float *,
                                   float *);
hipError_t launch_fft_conv(hipStream_t, const gf_batch *, const gf_psf *, const float *, int, float2 *, float2 *,
                           float *, const int *, const WorkView *, const Chi2Epi *ep = nullptr,
                           const FftFork *fork = nullptr);
hipError_t launch_fft_corr(hipStream_t, const gf_batch *, const gf_psf *, const float *, float2 *, float2 *, float *);
hipError_t launch_fft_otf(hipStream_t, const gf_batch *, const gf_psf *, const float *, const Work *, int,
                          const Work *, int, const int64_t *, float2 *, const int64_t *);
hipError_t launch_fft2d_otf(hipStream_t, const gf_batch *, const gf_psf *, const float *, const Work *, const int *);
hipError_t launch_direct(hipStream_t, const gf_batch *, const gf_psf *, const float *, int, float *, bool,
                         const int *, const WorkView *);
hipError_t launch_chi2(hipStream_t, const gf_batch *, const float *, const void *, bool, const float *,
                       const float *, float *, float2 *, unsigned int *, float2 *, const int *);
hipError_t launch_cot_prep(hipStream_t, const gf_batch *, const float *, const float *, float, float *, float2 *);
hipError_t launch_adjoint_final(hipStream_t, const gf_batch *, const int32_t *, const float *, const float2 *,
                                float *);
hipError_t launch_jac_assemble(hipStream_t, const gf_batch *, const float *, int, float *);
hipError_t launch_add_sky(hipStream_t, const gf_batch *, const float *, float *);
hipError_t launch_normal_eq(hipStream_t, const gf_batch *, const float *, const double *, const float *,
                            const float *, float *, int, int, const int *, const WorkView *, float2 *, int px = 0,
                            const float *mie = nullptr);
hipError_t launch_copy_runs(hipStream_t, const CopyRun *, int, Work *);
hipError_t launch_lm_init(hipStream_t, const gf_batch *, double, const int32_t *, const float2 *, LMState *, int *, int *,
                          int *, int model_ie = 0);
hipError_t launch_lm_start(hipStream_t, const gf_batch *, const double *, double *, const double *, const double *,
                           double *, int, const float4 *, CompC *);
hipError_t launch_lm_solve(hipStream_t, const gf_batch *, const float *, const gf_lm_opts *, LMState *, double *,
                           const double *, double *, int *, int *, int *, CompC *, CompC *, const float4 *,
                           const WorkView *, int px = 0);
hipError_t launch_chi2_direct(hipStream_t, const gf_batch *, const gf_psf *, const float *, const void *, bool,
                              const float *, const float *, float2 *, const int *, const WorkView *);
hipError_t launch_pair_final(hipStream_t, int, const int32_t *, const float2 *, float2 *, const int *);
hipError_t launch_lm_update(hipStream_t, const gf_batch *, const gf_lm_opts *, const int32_t *, const float2 *,
                            LMState *, double *, const double *, int *, int *, int *, CompC *, CompC *,
                            const WorkView *, int model_ie = 0);
hipError_t launch_lm_result(hipStream_t, int, const LMState *, gf_lm_result *);
hipError_t launch_group_best(hipStream_t, const gf_batch *, const gf_lm_result *, const double *, double *, int32_t *);
hipError_t launch_expand_starts(hipStream_t, int, int, const double *, double *);
hipError_t launch_nm_init(hipStream_t, const gf_batch *, const double *, const double *, const gf_simplex_opts *,
                          double *, double *, void *, int *, int *);
hipError_t launch_nm_step(hipStream_t, const gf_batch *, const int32_t *, const float2 *, const gf_simplex_opts *,
                          void *, double *, double *, double *, double *, int *, double *, int, int *);
hipError_t launch_nm_result(hipStream_t, const gf_batch *, const void *, const double *, const double *, double *,
                            gf_lm_result *);
hipError_t launch_nm_zero(hipStream_t, int *);
size_t nm_state_bytes();
hipError_t launch_mcmc_propose(hipStream_t, const gf_batch *, const double *, const double *, const double *,
                               const double *, uint64_t, uint64_t, uint64_t, int64_t, const int64_t *, double *, int *);
hipError_t launch_mcmc_init(hipStream_t, int, const float2 *, double *, int64_t *);
hipError_t launch_mcmc_accept(hipStream_t, const gf_batch *, const int32_t *, const float2 *, const int *, uint64_t,
                              uint64_t,
                              uint64_t, int64_t, int64_t *, double *, const double *, double *, int32_t *, float *,
                              int);
}  // namespace gf

using namespace gf;

namespace gf {
thread_local Profiler *t_prof = nullptr;

uint64_t next_uid() {
  static std::atomic<uint64_t> n{0};
  return ++n;
}
}

namespace {

gf_status fail(gf_ctx *c, gf_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

#define GF_TRY(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return fail(ctx, GF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t upload(T **d, const std::vector<T> &h) {
  *d = nullptr;
  if (h.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void **)d, h.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Bump allocator over the context workspace; run once with base == nullptr
// to size it.
struct Arena {
  char *base = nullptr;
  size_t off = 0;
  template <typename T>
  T *take(int64_t n) {
    const size_t a = (off + 255) & ~(size_t)255;
    off = a + (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    return base ? (T *)(base + a) : nullptr;
  }
};

gf_status ensure_ws(gf_ctx *c, size_t bytes) {
  if (bytes <= c->ws_bytes) return GF_OK;
  GF_TRY(c, hipStreamSynchronize(c->stream));
  dfree(c->ws);
  c->ws_bytes = 0;
  const size_t nb = bytes + bytes / 4;
  if (hipMalloc(&c->ws, nb) != hipSuccess) {
    c->ws = nullptr;
    return fail(c, GF_ENOMEM, "workspace allocation of " + std::to_string(nb) + " bytes failed");
  }
  c->ws_bytes = nb;
  return GF_OK;
}

gf_status ensure_counters(gf_ctx *c, int64_t n) {
  if (n <= c->n_counters) return GF_OK;
  GF_TRY(c, hipStreamSynchronize(c->stream));
  dfree(c->d_counters);
  c->n_counters = 0;
  const int64_t nn = std::max<int64_t>(n, 1024);
  if (hipMalloc((void **)&c->d_counters, nn * sizeof(unsigned int)) != hipSuccess)
    return fail(c, GF_ENOMEM, "counter allocation failed");
  GF_TRY(c, hipMemsetAsync(c->d_counters, 0, nn * sizeof(unsigned int), c->stream));
  GF_TRY(c, hipStreamSynchronize(c->stream));
  c->n_counters = nn;
  return GF_OK;
}

bool smooth(int v) {
  for (int p : {2, 3, 5})
    while (v % p == 0) v /= p;
  return v == 1;
}

// Smallest even 2^a 3^b 5^c >= m.
int fft_side(int m) {
  int L = std::max(m, 8);
  if (L & 1) ++L;
  while (!smooth(L)) L += 2;
  return L;
}

// Radices the LDS passes compute in registers.  A pass of radix R gives each
// of the 256 threads ceil(kFftCap / (256 R)) butterflies, so the busiest
// thread handles NB(R) R points; the plan is the factorisation of L that
// minimises the sum over passes of NB(R) R (1 + 0.15 log2 R) + 10 (the last
// term stands for a pass's two workgroup barriers).  For example 288 = 16 x 18
// (both passes keep 80-95 % of the threads busy) beats 32 x 9 (47 % busy in
// the first pass).
constexpr int kRadices[] = {32, 27, 25, 24, 20, 18, 16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};

double pass_cost(int R) {
  const int nb = (kFftCap + kThreads * R - 1) / (kThreads * R);
  return nb * R * (1.0 + 0.15 * std::log2((double)R)) + 10.0;
}

// Best factorisation of v into radices no larger than `maxr` (non-increasing
// order, so each multiset is visited once).
double best_plan(int v, int maxr, std::vector<int> &out) {
  if (v == 1) {
    out.clear();
    return 0.0;
  }
  double best = 1e300;
  std::vector<int> bestv, tmp;
  for (int r : kRadices) {
    if (r > maxr || v % r) continue;
    const double c = pass_cost(r) + best_plan(v / r, r, tmp);
    if (c < best) {
      best = c;
      bestv.assign(1, r);
      bestv.insert(bestv.end(), tmp.begin(), tmp.end());
    }
  }
  out = bestv;
  return best;
}

FftPlan make_plan(int L, int tw_off) {
  FftPlan p;
  std::memset(&p, 0, sizeof(p));
  p.L = L;
  p.tw_off = tw_off;
  std::vector<int> rad, rad18, rad24;
  best_plan(L, 32, rad);
  // A plan of radices up to 18 (else 24) runs in the FFT kernels built
  // without the larger butterflies (fewer registers, more waves per SIMD):
  // take it when it needs no more LDS passes than the best plan overall.
  best_plan(L, 18, rad18);
  best_plan(L, 24, rad24);
  if (!rad18.empty() && rad18.size() <= rad.size())
    rad = rad18;
  else if (!rad24.empty() && rad24.size() <= rad.size())
    rad = rad24;
  p.nstages = (int)rad.size();
  int ns = 1;
  for (int s = 0; s < p.nstages; ++s) {
    p.radix[s] = rad[s];
    p.ns[s] = ns;
    p.ns_magic[s] = magic_for((uint32_t)ns);
    p.nb_magic[s] = magic_for((uint32_t)(L / rad[s]));
    ns *= rad[s];
  }
  return p;
}


int padded_P(int nc) { return kNPC * nc + 1; }

// Longest-processing-time-first order of a launch list: the units of the
// costliest stamps are dispatched first, so the short ones fill the tail of
// the launch.  The order changes no result: every unit writes its own slot.
template <typename Key>
void lpt_order(std::vector<Work> &v, Key key) {
  std::stable_sort(v.begin(), v.end(), [&](const Work &a, const Work &b) { return key(a.stamp) > key(b.stamp); });
}

// Steps 2-3 for a one-channel padded model, chi^2 partials only: every stamp
// in mask gets its partials at p->d_c2_first (FFT stamps from the inverse-row
// pass, which writes no model image unless keep_model is set, and then only
// for one-component stamps; direct stamps from the direct convolution into
// mconv and the chi^2 kernel).  With keep_model, mconv holds the convolved
// model of every one-component stamp in mask afterwards.
hipError_t conv_chi2(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *mpad, float2 *S1, float2 *S2,
                     float *mconv, const void *theta, bool theta_f64, const float *data, const float *weight,
                     float2 *part, const int *mask, const WorkView *v, const FftFork *fork, bool keep_model = false) {
  Chi2Epi ep{data, weight, theta, theta_f64 ? 1 : 0, p->d_c2_first, part};
  if (keep_model) ep.model = mconv;
  hipError_t e = launch_fft_conv(st, b, p, mpad, 1, S1, S2, mconv, mask, v, &ep, fork);
  if (e == hipSuccess) e = launch_direct(st, b, p, mpad, 1, mconv, false, mask, v);
  if (e == hipSuccess) e = launch_chi2_direct(st, b, p, mconv, theta, theta_f64, data, weight, part, mask, v);
  return e;
}

// Partial slots of a chi^2 buffer that serves both layouts (per kPixChunk
// pixels and per conv_chi2 slot).
int64_t chi2_slots(const gf_batch *b, const gf_psf *p) { return std::max<int64_t>((int64_t)b->h_pix.size(), p->n_c2); }

}  // namespace

extern "C" {

const char *gf_version(void) { return "libgf 0.2 (gfx950)"; }

static void fork_destroy(FftFork &f) {
  for (int i = 0; i < kForkLanes; ++i) {
    if (f.side[i]) (void)hipStreamDestroy(f.side[i]);
    if (f.join[i]) (void)hipEventDestroy(f.join[i]);
  }
  if (f.fork) (void)hipEventDestroy(f.fork);
  f = FftFork{};
}

gf_status gf_create(gf_ctx **out, int device, const char *autotune_cache) {
  if (!out) return GF_EINVAL;
  *out = nullptr;
  gf_ctx *c = new (std::nothrow) gf_ctx();
  if (!c) return GF_ENOMEM;
  c->device = device;
  if (autotune_cache) c->tune_path = autotune_cache;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return GF_EDEVICE;
  }
  std::vector<float4> tab = build_bn_table();
  if (upload(&c->d_bn, tab) != hipSuccess) {
    delete c;
    return GF_EDEVICE;
  }
  if (hipHostMalloc((void **)&c->h_pinned, sizeof(int) * 8 * std::max(2, kLmLanes), hipHostMallocDefault) != hipSuccess) {
    dfree(c->d_bn);
    delete c;
    return GF_ENOMEM;
  }
  if (ensure_counters(c, 1024) != GF_OK) {
    dfree(c->d_bn);
    (void)hipHostFree(c->h_pinned);
    delete c;
    return GF_ENOMEM;
  }
  if (!c->tune_path.empty()) (void)tune_load(c);   // an unreadable or foreign table is ignored
  bool fork_ok = hipEventCreateWithFlags(&c->fork.fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < kForkLanes && fork_ok; ++i)
    fork_ok = hipStreamCreateWithFlags(&c->fork.side[i], hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->fork.join[i], hipEventDisableTiming) == hipSuccess;
  if (!fork_ok || noalloc_init(device) != hipSuccess) {
    fork_destroy(c->fork);
    dfree(c->d_bn);
    dfree(c->d_counters);
    (void)hipHostFree(c->h_pinned);
    delete c;
    return GF_EDEVICE;
  }
  *out = c;
  return GF_OK;
}

// Wait for everything the context has enqueued, on its own streams only, so
// that contexts used by other host threads (possibly capturing graphs) are
// not touched.
static void ctx_sync(gf_ctx *c) {
  (void)hipStreamSynchronize(c->stream);
  for (hipStream_t s : {c->lm_stream, c->fork.side[0], c->fork.side[1], c->fork.side[2]})
    if (s) (void)hipStreamSynchronize(s);
  for (hipStream_t s : c->lm_lane_stream)
    if (s) (void)hipStreamSynchronize(s);
  for (hipStream_t s : c->side)
    if (s) (void)hipStreamSynchronize(s);
}

void gf_destroy(gf_ctx *c) {
  if (!c) return;
  ctx_sync(c);
  dfree(c->d_bn);
  dfree(c->d_counters);
  dfree(c->ws);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->h_states) (void)hipHostFree(c->h_states);
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  for (hipStream_t st : c->side)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t e : c->side_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->lm_exec) (void)hipGraphExecDestroy(c->lm_exec);
  if (c->lm_graph) (void)hipGraphDestroy(c->lm_graph);
  if (c->lm_stream) (void)hipStreamDestroy(c->lm_stream);
  if (c->lm_ev) (void)hipEventDestroy(c->lm_ev);
  for (hipStream_t s : c->lm_lane_stream)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : c->lm_lane_ev)
    if (e) (void)hipEventDestroy(e);
  fork_destroy(c->fork);
  delete c;
}

int gf_tune_form_get(const gf_ctx *c, int L) {
  const int k = c ? f2d_class(L) : -1;
  return k < 0 ? 0 : c->tune_form[k];
}

gf_status gf_tune_form_set(gf_ctx *c, int L, int form) {
  if (!c) return GF_EINVAL;
  const int k = f2d_class(L);
  if (k < 0 || !(form == -1 || form == 1 || form == 2))
    return fail(c, GF_EINVAL, "gf_tune_form_set: L is not a one-workgroup side or form is not -1, 1 or 2");
  c->tune_form[k] = (int8_t)form;
  return GF_OK;
}

int gf_tune_direct_get(const gf_ctx *c) { return c ? c->tune_direct_k : 0; }

gf_status gf_tune_direct_set(gf_ctx *c, int k) {
  if (!c || k < 1 || k > GF_MAX_K || (k % 2) == 0) return fail(c, GF_EINVAL, "gf_tune_direct_set: odd K in 1..GF_MAX_K");
  c->tune_direct_k = k;
  c->tune_direct_done = 1;
  (void)tune_save(c);
  return GF_OK;
}

int gf_tune_min_active_get(const gf_ctx *c, int L) {
  const int k = c ? f2d_class(L) : -1;
  return k < 0 ? -1 : c->f2d_min_active[f2d_bucket(k)];
}

gf_status gf_tune_min_active_set(gf_ctx *c, int L, int n) {
  if (!c) return GF_EINVAL;
  const int k = f2d_class(L);
  if (k < 0 || n < 0) return fail(c, GF_EINVAL, "gf_tune_min_active_set: L is not a one-workgroup side or n < 0");
  c->f2d_min_active[f2d_bucket(k)] = n;
  c->tune_min_done[f2d_bucket(k)] = 1;
  return GF_OK;
}

gf_status gf_set_stream(gf_ctx *c, void *stream) {
  if (!c) return GF_EINVAL;
  c->stream = (hipStream_t)stream;
  return GF_OK;
}

const char *gf_last_error(const gf_ctx *c) { return c ? c->err.c_str() : "null context"; }

gf_status gf_synchronize(gf_ctx *c) {
  if (!c) return GF_EINVAL;
  GF_TRY(c, hipStreamSynchronize(c->stream));
  return GF_OK;
}

// ------------------------------------------------------------------ batches
// flat_P > 0: stamps that are flat arrays of H*W values with flat_P
// parameters each (a data cube's voxels for chi^2, the normal equations and
// the LM state); no convolution runs on them, so the FFT size limit does not
// apply.
static gf_status create_batch(gf_ctx *c, int n, const int32_t *H, const int32_t *W, const int32_t *K,
                              const int32_t *nc, int shared, const int32_t *group, gf_batch **out, int flat_P = 0) {
  if (!c || !out || !H || !W || !K || !nc || n <= 0) return fail(c, GF_EINVAL, "gf_batch_create: bad argument");
  *out = nullptr;
  // groups: every stamp's observation and PSF, or one per group
  int G = 0;
  std::vector<int> gfirst_stamp;
  if (group) {
    for (int s = 0; s < n; ++s) {
      if (group[s] < 0 || group[s] >= n) return fail(c, GF_EINVAL, "gf_batch_create_grouped: group id out of range");
      G = std::max(G, group[s] + 1);
    }
    gfirst_stamp.assign(G, -1);
    for (int s = 0; s < n; ++s) {
      int &f = gfirst_stamp[group[s]];
      if (f < 0) {
        f = s;
      } else if (H[s] != H[f] || W[s] != W[f] || K[s] != K[f]) {
        return fail(c, GF_ESHAPE, "gf_batch_create_grouped: stamps of a group need the same H, W and K");
      }
    }
    for (int g = 0; g < G; ++g)
      if (gfirst_stamp[g] < 0) return fail(c, GF_EINVAL, "gf_batch_create_grouped: group ids must be 0 .. G-1, all used");
  }
  gf_batch *b = new (std::nothrow) gf_batch();
  if (!b) return fail(c, GF_ENOMEM, "gf_batch_create: host allocation");
  b->ctx = c;
  b->uid = next_uid();
  b->n = n;
  b->shared = shared != 0;
  b->h_desc.resize(n);
  int64_t pix = 0, pad = 0, psf = 0, par = 0, jac = 0;
  std::vector<int64_t> gimg(G, 0), gpsf(G, 0);
  int64_t gi = 0, gp = 0;
  for (int g = 0; g < G; ++g) {
    const int f = gfirst_stamp[g];
    gimg[g] = gi;
    gpsf[g] = gp;
    gi += (int64_t)H[f] * W[f];
    gp += (int64_t)K[f] * K[f];
  }
  for (int s = 0; s < n; ++s) {
    const bool fft_ok = flat_P > 0 ? K[s] == 1 && nc[s] == 1 && (int64_t)H[s] * W[s] <= (1LL << 30)
                                   : H[s] + K[s] - 1 <= GF_MAX_FFT && W[s] + K[s] - 1 <= GF_MAX_FFT;
    if (H[s] <= 0 || W[s] <= 0 || K[s] <= 0 || (K[s] % 2) == 0 || K[s] > GF_MAX_K || nc[s] < 1 ||
        nc[s] > GF_MAX_COMP || !fft_ok) {
      delete b;
      return fail(c, GF_ESHAPE, "gf_batch_create: unsupported shape for stamp " + std::to_string(s));
    }
    if (b->shared && (H[s] != H[0] || W[s] != W[0] || K[s] != K[0] || nc[s] != nc[0])) {
      delete b;
      return fail(c, GF_ESHAPE, "gf_batch_create: shared-image batch needs identical stamps");
    }
    StampDesc &d = b->h_desc[s];
    d.H = H[s];
    d.W = W[s];
    d.K = K[s];
    d.ncomp = nc[s];
    d.Mh = H[s] + K[s] - 1;
    d.Mw = W[s] + K[s] - 1;
    d.P = flat_P > 0 ? flat_P : padded_P(nc[s]);
    d.pad0 = 0;
    d.pix = pix;
    d.pad = pad;
    d.par = par;
    d.jac = jac;
    d.img = b->shared ? 0 : group ? gimg[group[s]] : pix;
    d.psf = b->shared ? 0 : group ? gpsf[group[s]] : psf;
    pix += (int64_t)d.H * d.W;
    pad += (int64_t)d.Mh * d.Mw;
    psf += (int64_t)d.K * d.K;
    par += d.P;
    jac += (int64_t)d.P * d.H * d.W;
    b->max_nc = std::max(b->max_nc, d.ncomp);
    b->max_P = std::max(b->max_P, d.P);
    if (s > 0 && (d.H != H[0] || d.W != W[0] || d.K != K[0] || d.ncomp != nc[0])) b->uniform = false;
  }
  b->n_pix = pix;
  b->n_pad = pad;
  b->n_psf = b->shared ? (int64_t)K[0] * K[0] : group ? gp : psf;
  b->n_par = par;
  b->n_img = b->shared ? (int64_t)H[0] * W[0] : group ? gi : pix;
  // group membership lists (stamps in increasing order within a group)
  b->n_groups = group ? G : (b->shared ? 1 : n);
  {
    std::vector<int32_t> cnt(b->n_groups + 1, 0);
    for (int s = 0; s < n; ++s) cnt[(group ? group[s] : b->shared ? 0 : s) + 1] += 1;
    for (int g = 0; g < b->n_groups; ++g) cnt[g + 1] += cnt[g];
    b->h_gfirst = cnt;
    b->h_gmembers.assign(n, 0);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int s = 0; s < n; ++s) b->h_gmembers[fill[group ? group[s] : b->shared ? 0 : s]++] = s;
  }
  b->n_jac = jac;
  for (int s = 0; s < n; ++s) {
    const StampDesc &d = b->h_desc[s];
    b->h_eval_first.push_back((int32_t)b->h_eval.size());
    const int ne = (d.Mh * d.Mw + kEvalTile - 1) / kEvalTile;
    for (int u = 0; u < ne; ++u) b->h_eval.push_back({s, u});
    b->h_pix_first.push_back((int32_t)b->h_pix.size());
    const int np = (d.H * d.W + kPixChunk - 1) / kPixChunk;
    for (int u = 0; u < np; ++u) b->h_pix.push_back({s, u});
    b->h_neq_first.push_back((int32_t)b->h_neq.size());
    const int nq = (d.H * d.W + kNeqChunk - 1) / kNeqChunk;
    for (int u = 0; u < nq; ++u) b->h_neq.push_back({s, u});
  }
  // launch order: the largest stamps first (so the units of the stamps of
  // at least kNeqBigPix pixels, the eight-wave workgroups, lead the list)
  auto npad = [&](int s) { return (int64_t)b->h_desc[s].Mh * b->h_desc[s].Mw; };
  auto npx = [&](int s) { return (int64_t)b->h_desc[s].H * b->h_desc[s].W; };
  lpt_order(b->h_eval, npad);
  lpt_order(b->h_pix, npx);
  lpt_order(b->h_neq, npx);
  for (const Work &w : b->h_neq) b->n_neq_big += b->h_desc[w.stamp].H * b->h_desc[w.stamp].W >= kNeqBigPix;
  b->h_eval_first.push_back((int32_t)b->h_eval.size());
  b->h_pix_first.push_back((int32_t)b->h_pix.size());
  b->h_neq_first.push_back((int32_t)b->h_neq.size());
  if (b->h_eval.size() > 0x7fffffffu) {
    delete b;
    return fail(c, GF_ESHAPE, "gf_batch_create: batch too large");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&b->d_desc, b->h_desc);
  if (e == hipSuccess) e = upload(&b->d_eval, b->h_eval);
  if (e == hipSuccess) e = upload(&b->d_pix, b->h_pix);
  if (e == hipSuccess) e = upload(&b->d_neq, b->h_neq);
  if (e == hipSuccess) e = upload(&b->d_pix_first, b->h_pix_first);
  if (e == hipSuccess) e = upload(&b->d_neq_first, b->h_neq_first);
  if (e == hipSuccess) e = upload(&b->d_eval_first, b->h_eval_first);
  if (e == hipSuccess) e = upload(&b->d_gfirst, b->h_gfirst);
  if (e == hipSuccess) e = upload(&b->d_gmembers, b->h_gmembers);
  if (e == hipSuccess) e = hipMalloc(&b->d_cc, sizeof(gf::CompC) * (size_t)b->n * kMaxComp);
  if (e != hipSuccess) {
    gf_batch_destroy(b);
    return fail(c, GF_EDEVICE, std::string("gf_batch_create: ") + hipGetErrorString(e));
  }
  *out = b;
  return GF_OK;
}

gf_status gf_batch_create(gf_ctx *c, int n, const int32_t *H, const int32_t *W, const int32_t *K,
                          const int32_t *nc, int shared, gf_batch **out) {
  return create_batch(c, n, H, W, K, nc, shared, nullptr, out);
}

gf_status gf_batch_create_grouped(gf_ctx *c, int n, const int32_t *H, const int32_t *W, const int32_t *K,
                                  const int32_t *nc, const int32_t *group, gf_batch **out) {
  if (!group) return fail(c, GF_EINVAL, "gf_batch_create_grouped: null group array");
  return create_batch(c, n, H, W, K, nc, 0, group, out);
}

void gf_batch_destroy(gf_batch *b) {
  if (!b) return;
  dfree(b->d_desc);
  dfree(b->d_eval);
  dfree(b->d_pix);
  dfree(b->d_neq);
  dfree(b->d_pix_first);
  dfree(b->d_neq_first);
  dfree(b->d_eval_first);
  dfree(b->d_gfirst);
  dfree(b->d_gmembers);
  dfree(b->d_cc);
  delete b;
}

int gf_batch_count(const gf_batch *b) { return b ? b->n : 0; }

gf_status gf_batch_sizes(const gf_batch *b, int64_t *n_pix, int64_t *n_pad, int64_t *n_psf, int64_t *n_par,
                         int64_t *n_img, int64_t *n_jac) {
  if (!b) return GF_EINVAL;
  if (n_pix) *n_pix = b->n_pix;
  if (n_pad) *n_pad = b->n_pad;
  if (n_psf) *n_psf = b->n_psf;
  if (n_par) *n_par = b->n_par;
  if (n_img) *n_img = b->n_img;
  if (n_jac) *n_jac = b->n_jac;
  return GF_OK;
}

gf_status gf_batch_offsets(const gf_batch *b, int64_t *pix, int64_t *pad, int64_t *psf, int64_t *par, int64_t *img,
                           int64_t *jac) {
  if (!b) return GF_EINVAL;
  for (int s = 0; s < b->n; ++s) {
    const StampDesc &d = b->h_desc[s];
    if (pix) pix[s] = d.pix;
    if (pad) pad[s] = d.pad;
    if (psf) psf[s] = d.psf;
    if (par) par[s] = d.par;
    if (img) img[s] = d.img;
    if (jac) jac[s] = d.jac;
  }
  return GF_OK;
}

// ---------------------------------------------------------------------- PSF
gf_status gf_psf_prepare(gf_ctx *c, const gf_batch *b, const float *taps, int mode, gf_psf **out) {
  if (!c || !b || !taps || !out || mode < GF_CONV_AUTO || mode > GF_CONV_FFT_FUSED)
    return fail(c, GF_EINVAL, "gf_psf_prepare: bad argument");
  *out = nullptr;
  // first use of a one-workgroup side by the automatic choice of a context
  // with a tuning file: measure it now
  if (mode == GF_CONV_AUTO && !c->tune_path.empty()) {
    if (!c->tune_direct_done) {
      bool near = false;   // a PSF side where the direct-path threshold decides
      for (const StampDesc &d : b->h_desc) near |= d.K >= 3 && d.K <= 15;
      if (near) {
        const gf_status ts = tune_direct(c);
        if (ts != GF_OK) return fail(c, ts, "gf_psf_prepare: measuring the direct-path threshold failed");
      }
    }
    std::vector<char> seen(kF2dN, 0);
    for (const StampDesc &d : b->h_desc) {
      const int k = d.K > c->tune_direct_k ? f2d_class(fft_side(std::max(d.Mh, d.Mw))) : -1;
      if (k < 0 || seen[k] || c->tune_form[k] >= 0) continue;
      seen[k] = 1;
      const gf_status ts = tune_side(c, kF2dSides[k]);
      if (ts != GF_OK) return fail(c, ts, "gf_psf_prepare: measuring the FFT forms of side " +
                                              std::to_string(kF2dSides[k]) + " failed");
    }
  }
  gf_psf *p = new (std::nothrow) gf_psf();
  if (!p) return fail(c, GF_ENOMEM, "gf_psf_prepare: host allocation");
  p->ctx = c;
  p->uid = next_uid();
  p->batch = b;
  p->d_taps = taps;
  const int n = b->n;
  p->h_path.resize(n);
  p->h_s1.assign(n, 0);
  p->h_s2.assign(n, 0);
  p->h_s1a.assign(n, 0);
  p->h_s2a.assign(n, 0);
  std::vector<int> plan_of_L(GF_MAX_FFT + 1, -1);
  std::vector<float2> tw;
  std::vector<int64_t> otf_tmp(n, 0), otf_off(n, 0);
  std::map<int64_t, int64_t> otf_of_psf;   // PSF offset -> OTF offset (the layout of the stamp's form)
  std::map<int64_t, int64_t> otf_mp_of_psf;   // PSF offset -> bin-major OTF offset
  std::vector<Work> otf_rows, otf_cols;
  std::vector<Work> f2d_cls[kF2dN], f2d_otf_cls[kF2dN];
  int64_t otf_tmp_n = 0;
  // Path of each stamp: 0 direct, 1 multi-pass FFT, 2 one-workgroup FFT.
  // Automatic choice: the direct sum costs about K^2 FMAs per output pixel
  // and channel (K = 15: ~32 ps per pixel-channel measured), the FFT path a
  // roughly K-independent ~7-10 ps, so the FFT wins from K = 9 on; of the two
  // FFT forms the one-workgroup one is taken where the side allows it unless
  // the context's tuning table names the multi-pass form for that side.
  auto path_of = [&](const StampDesc &d) -> int {
    const int L = fft_side(std::max(d.Mh, d.Mw));
    const bool fits = f2d_class(L) >= 0;
    if (mode == GF_CONV_DIRECT) return d.K > kDirectMaxK ? 1 : 0;
    if (mode == GF_CONV_FFT_MULTIPASS) return 1;
    if (mode == GF_CONV_FFT_FUSED) return 2;
    if (mode == GF_CONV_AUTO && d.K <= c->tune_direct_k) return 0;
    if (!fits) return 1;
    if (mode == GF_CONV_AUTO) {
      // untuned sides: the one-workgroup form up to 160 (above, its kernels
      // run out of registers and the multi-pass form is faster)
      const int f = c->tune_form[f2d_class(L)];
      if (f > 0) return f;
      return L <= 160 ? 2 : 1;
    }
    return 2;
  };
  // The largest radix over the plans of the multi-pass stamps picks the
  // kernel build and with it the LDS capacity that sizes every work unit.
  {
    std::vector<char> seen(GF_MAX_FFT + 1, 0);
    for (int s = 0; s < n; ++s) {
      const StampDesc &d = b->h_desc[s];
      const bool f = path_of(d) != 0;   // one-workgroup stamps may run multi-pass too
      const int L = fft_side(std::max(d.Mh, d.Mw));
      if (!f || L > GF_MAX_FFT || seen[L]) continue;
      seen[L] = 1;
      const FftPlan pl = make_plan(L, 0);
      for (int q = 0; q < pl.nstages; ++q)
        p->rmax = std::max(p->rmax, pl.radix[q] <= 18 ? 18 : pl.radix[q] <= 24 ? 24 : 32);
    }
  }
  const int cap = fft_cap(p->rmax);
  for (int s = 0; s < n; ++s) {
    const StampDesc &d = b->h_desc[s];
    int path = path_of(d);
    if (mode == GF_CONV_DIRECT && d.K > kDirectMaxK) {
      delete p;
      return fail(c, GF_ESHAPE, "gf_psf_prepare: PSF too large for the direct path");
    }
    const bool fft = path != 0;
    if (path == 2 && f2d_class(fft_side(std::max(d.Mh, d.Mw))) < 0) {
      delete p;
      return fail(c, GF_ESHAPE, "gf_psf_prepare: padded grid exceeds the one-workgroup FFT side");
    }
    PathDesc &pd = p->h_path[s];
    pd.fft = path;
    pd.L = 0;
    pd.plan = -1;
    pd.tw = 0;
    pd.otf = 0;
    pd.otf_mp = 0;
    p->h_c2_first.push_back((int32_t)p->n_c2);
    if (!fft) {
      const int np = (d.H * d.W + kPixChunk - 1) / kPixChunk;
      for (int u = 0; u < np; ++u) p->h_pix_direct.push_back({s, u});
      p->n_c2 += np;
    } else {
      p->n_c2 += (d.H + 1) / 2;
    }
    if (!fft) {
      ++p->n_direct;
      const int tx = (d.W + kDirectTW - 1) / kDirectTW, ty = (d.H + kDirectTH - 1) / kDirectTH;
      for (int u = 0; u < tx * ty; ++u) p->h_direct.push_back({s, u});
      const int ax = (d.Mw + kDirectTW - 1) / kDirectTW, ay = (d.Mh + kDirectTH - 1) / kDirectTH;
      for (int u = 0; u < ax * ay; ++u) p->h_adirect.push_back({s, u});
      continue;
    }
    ++p->n_fft;
    const int L = fft_side(std::max(d.Mh, d.Mw));
    if (L > GF_MAX_FFT) {
      delete p;
      return fail(c, GF_ESHAPE, "gf_psf_prepare: padded grid exceeds the largest FFT side");
    }
    if (plan_of_L[L] < 0) {
      plan_of_L[L] = (int)p->h_plans.size();
      p->h_plans.push_back(make_plan(L, (int)tw.size()));
      for (int k = 0; k < L; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)L;
        tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
      }
    }
    p->max_L = std::max(p->max_L, L);
    pd.L = L;
    pd.plan = plan_of_L[L];
    pd.tw = p->h_plans[pd.plan].tw_off;
    const int Lh = L / 2 + 1;
    const bool f2 = path == 2;
    if (f2) {
      const int cls = f2d_class(L);
      ++p->n_f2d;
      f2d_cls[cls].push_back({s, f2d_bucket(cls)});
      auto hit = otf_of_psf.find(d.psf);
      if (hit == otf_of_psf.end()) {
        otf_of_psf[d.psf] = p->n_otf;
        pd.otf = p->n_otf;
        p->n_otf += (int64_t)L * Lh;
        f2d_otf_cls[cls].push_back({s, f2d_bucket(cls)});
      } else {
        pd.otf = hit->second;
      }
    }
    // multi-pass units (for a one-workgroup stamp: the alternative used
    // once few of its bucket's stamps are still fitting)
    const int T = cap / (L + 1), C = cap / L;
    const int cols = (Lh + C - 1) / C;
    for (int u = 0; u < (d.Mh + 2 * T - 1) / (2 * T); ++u) (f2 ? p->h_rows_alt : p->h_rows).push_back({s, u});
    for (int u = 0; u < cols; ++u) (f2 ? p->h_cols_alt : p->h_cols).push_back({s, u});
    for (int u = 0; u < (d.H + 2 * T - 1) / (2 * T); ++u) (f2 ? p->h_irows_alt : p->h_irows).push_back({s, u});
    if (!f2) {
      for (int u = 0; u < (d.H + 2 * T - 1) / (2 * T); ++u) p->h_arows.push_back({s, u});
      for (int u = 0; u < cols; ++u) p->h_acols.push_back({s, u});
      for (int u = 0; u < (d.Mh + 2 * T - 1) / (2 * T); ++u) p->h_airows.push_back({s, u});
      p->h_s1a[s] = p->n_s1a;
      p->n_s1a += (int64_t)d.H * Lh;
      p->h_s2a[s] = p->n_s2a;
      p->n_s2a += (int64_t)d.Mh * Lh;
    }
    {
      const int Tn = std::min(T, kFftNarrowT), Cn = std::min(C, kFftNarrowC);
      for (int u = 0; u < (d.Mh + 2 * Tn - 1) / (2 * Tn); ++u)
        (f2 ? p->h_rows_n_alt : p->h_rows_n).push_back({s, u});
      for (int u = 0; u < (Lh + Cn - 1) / Cn; ++u) (f2 ? p->h_cols_n_alt : p->h_cols_n).push_back({s, u});
      for (int u = 0; u < (d.H + 2 * Tn - 1) / (2 * Tn); ++u)
        (f2 ? p->h_irows_n_alt : p->h_irows_n).push_back({s, u});
    }
    p->h_s1[s] = p->n_s1;
    p->n_s1 += (int64_t)d.Mh * Lh;
    p->h_s2[s] = p->n_s2;
    p->n_s2 += (int64_t)d.H * Lh;
    auto hit = otf_mp_of_psf.find(d.psf);
    if (hit == otf_mp_of_psf.end()) {
      otf_mp_of_psf[d.psf] = p->n_otf;
      otf_off[s] = p->n_otf;
      pd.otf_mp = p->n_otf;
      p->n_otf += (int64_t)L * Lh;
      otf_tmp[s] = otf_tmp_n;
      otf_tmp_n += (int64_t)d.K * Lh;
      for (int u = 0; u < (d.K + 2 * T - 1) / (2 * T); ++u) otf_rows.push_back({s, u});
      for (int u = 0; u < cols; ++u) otf_cols.push_back({s, u});
    } else {
      pd.otf_mp = hit->second;   // stamps sharing a PSF (same group) share its OTF
    }
    if (!f2) pd.otf = pd.otf_mp;
  }
  p->h_c2_first.push_back((int32_t)p->n_c2);
  if (p->n_c2 > 0x7fffffff) {
    delete p;
    return fail(c, GF_ESHAPE, "gf_psf_prepare: batch too large");
  }
  // launch lists in longest-first order (the multi-pass units by FFT side,
  // direct tiles by PSF side; within each one-workgroup bucket the largest
  // side first)
  {
    auto side = [&](int s) { return (int64_t)p->h_path[s].L; };
    auto ksz = [&](int s) { return (int64_t)b->h_desc[s].K; };
    for (auto *l : {&p->h_rows, &p->h_cols, &p->h_irows, &p->h_arows, &p->h_acols, &p->h_airows, &p->h_rows_n,
                    &p->h_cols_n, &p->h_irows_n, &p->h_rows_alt, &p->h_cols_alt, &p->h_irows_alt,
                    &p->h_rows_n_alt, &p->h_cols_n_alt, &p->h_irows_n_alt})
      lpt_order(*l, side);
    lpt_order(p->h_direct, ksz);
    lpt_order(p->h_adirect, ksz);
    lpt_order(p->h_pix_direct, ksz);
  }
  std::vector<Work> f2d_otf;
  int f2d_otf_first[kF2dBuckets + 1] = {};
  for (int bk = 0; bk < kF2dBuckets; ++bk) {
    p->f2d_first[bk] = (int)p->h_f2d.size();
    f2d_otf_first[bk] = (int)f2d_otf.size();
    for (int k = kF2dN - 1; k >= 0; --k) {
      if (f2d_bucket(k) != bk) continue;
      p->h_f2d.insert(p->h_f2d.end(), f2d_cls[k].begin(), f2d_cls[k].end());
      f2d_otf.insert(f2d_otf.end(), f2d_otf_cls[k].begin(), f2d_otf_cls[k].end());
    }
  }
  p->f2d_first[kF2dBuckets] = (int)p->h_f2d.size();
  f2d_otf_first[kF2dBuckets] = (int)f2d_otf.size();
  hipError_t e = hipSuccess;
  Work *d_orows = nullptr, *d_ocols = nullptr, *d_o2d = nullptr;
  int64_t *d_otmp = nullptr, *d_ooff = nullptr;
  if (e == hipSuccess) e = upload(&p->d_path, p->h_path);
  if (e == hipSuccess) e = upload(&p->d_plans, p->h_plans);
  if (e == hipSuccess) e = upload(&p->d_tw, tw);
  if (e == hipSuccess) e = upload(&p->d_rows, p->h_rows);
  if (e == hipSuccess) e = upload(&p->d_cols, p->h_cols);
  if (e == hipSuccess) e = upload(&p->d_irows, p->h_irows);
  if (e == hipSuccess) e = upload(&p->d_arows, p->h_arows);
  if (e == hipSuccess) e = upload(&p->d_acols, p->h_acols);
  if (e == hipSuccess) e = upload(&p->d_airows, p->h_airows);
  if (e == hipSuccess) e = upload(&p->d_rows_n, p->h_rows_n);
  if (e == hipSuccess) e = upload(&p->d_cols_n, p->h_cols_n);
  if (e == hipSuccess) e = upload(&p->d_irows_n, p->h_irows_n);
  if (e == hipSuccess) e = upload(&p->d_s1, p->h_s1);
  if (e == hipSuccess) e = upload(&p->d_s2, p->h_s2);
  if (e == hipSuccess) e = upload(&p->d_s1a, p->h_s1a);
  if (e == hipSuccess) e = upload(&p->d_s2a, p->h_s2a);
  if (e == hipSuccess) e = upload(&p->d_direct, p->h_direct);
  if (e == hipSuccess) e = upload(&p->d_adirect, p->h_adirect);
  if (e == hipSuccess) e = upload(&p->d_c2_first, p->h_c2_first);
  if (e == hipSuccess) e = upload(&p->d_pix_direct, p->h_pix_direct);
  if (e == hipSuccess) e = upload(&d_orows, otf_rows);
  if (e == hipSuccess) e = upload(&d_ocols, otf_cols);
  if (e == hipSuccess) e = upload(&d_otmp, otf_tmp);
  if (e == hipSuccess) e = upload(&d_ooff, otf_off);
  if (e == hipSuccess) e = upload(&p->d_f2d, p->h_f2d);
  if (e == hipSuccess) e = upload(&p->d_rows_alt, p->h_rows_alt);
  if (e == hipSuccess) e = upload(&p->d_cols_alt, p->h_cols_alt);
  if (e == hipSuccess) e = upload(&p->d_irows_alt, p->h_irows_alt);
  if (e == hipSuccess) e = upload(&p->d_rows_n_alt, p->h_rows_n_alt);
  if (e == hipSuccess) e = upload(&p->d_cols_n_alt, p->h_cols_n_alt);
  if (e == hipSuccess) e = upload(&p->d_irows_n_alt, p->h_irows_n_alt);
  if (e == hipSuccess) e = upload(&d_o2d, f2d_otf);
  if (e == hipSuccess && p->n_otf > 0) e = hipMalloc((void **)&p->d_otf, p->n_otf * sizeof(float2));
  if (e != hipSuccess) {
    dfree(d_o2d);
    dfree(d_orows);
    dfree(d_ocols);
    dfree(d_otmp);
    dfree(d_ooff);
    gf_psf_destroy(p);
    return fail(c, GF_EDEVICE, std::string("gf_psf_prepare: ") + hipGetErrorString(e));
  }
  gf_status st = GF_OK;
  if (!otf_rows.empty()) {
    st = ensure_ws(c, (size_t)otf_tmp_n * sizeof(float2) + 256);
    if (st == GF_OK) {
      e = launch_fft_otf(c->stream, b, p, taps, d_orows, (int)otf_rows.size(), d_ocols, (int)otf_cols.size(),
                         d_otmp, (float2 *)c->ws, d_ooff);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) st = fail(c, GF_EDEVICE, std::string("gf_psf_prepare (OTF): ") + hipGetErrorString(e));
    }
  }
  if (st == GF_OK && !f2d_otf.empty()) {
    e = launch_fft2d_otf(c->stream, b, p, taps, d_o2d, f2d_otf_first);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(c, GF_EDEVICE, std::string("gf_psf_prepare (OTF): ") + hipGetErrorString(e));
  }
  dfree(d_o2d);
  dfree(d_orows);
  dfree(d_ocols);
  dfree(d_otmp);
  dfree(d_ooff);
  if (st != GF_OK) {
    gf_psf_destroy(p);
    return st;
  }
  *out = p;
  return GF_OK;
}

void gf_psf_destroy(gf_psf *p) {
  if (!p) return;
  dfree(p->d_path);
  dfree(p->d_plans);
  dfree(p->d_tw);
  dfree(p->d_otf);
  dfree(p->d_rows);
  dfree(p->d_cols);
  dfree(p->d_irows);
  dfree(p->d_arows);
  dfree(p->d_acols);
  dfree(p->d_airows);
  dfree(p->d_rows_n);
  dfree(p->d_cols_n);
  dfree(p->d_irows_n);
  dfree(p->d_s1);
  dfree(p->d_s2);
  dfree(p->d_s1a);
  dfree(p->d_s2a);
  dfree(p->d_direct);
  dfree(p->d_adirect);
  dfree(p->d_c2_first);
  dfree(p->d_pix_direct);
  dfree(p->d_f2d);
  dfree(p->d_rows_alt);
  dfree(p->d_cols_alt);
  dfree(p->d_irows_alt);
  dfree(p->d_rows_n_alt);
  dfree(p->d_cols_n_alt);
  dfree(p->d_irows_n_alt);
  delete p;
}

gf_status gf_psf_paths(const gf_psf *p, int32_t *uses_fft, int32_t *side) {
  if (!p) return GF_EINVAL;
  for (size_t s = 0; s < p->h_path.size(); ++s) {
    if (uses_fft) uses_fft[s] = p->h_path[s].fft;
    if (side) side[s] = p->h_path[s].L;
  }
  return GF_OK;
}

// ------------------------------------------------------------ steps 1-3
gf_status gf_eval_model(gf_ctx *c, const gf_batch *b, const float *theta, int S, float *out) {
  ProfBind pb_(c);
  if (!c || !b || !theta || !out) return fail(c, GF_EINVAL, "gf_eval_model: null argument");
  if (b->ctx != c) return fail(c, GF_EINVAL, "gf_eval_model: batch belongs to another context");
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return fail(c, GF_EINVAL, "gf_eval_model: oversample out of range");
  GF_TRY(c, launch_eval(c->stream, b, theta, S, c->d_bn, out, nullptr));
  return GF_OK;
}

static gf_status convolve(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *in, int n_ch, float *out,
                          float2 *S1, float2 *S2, const int *mask) {
  GF_TRY(c, launch_fft_conv(c->stream, b, p, in, n_ch, S1, S2, out, mask, nullptr, nullptr, &c->fork));
  GF_TRY(c, launch_direct(c->stream, b, p, in, n_ch, out, false, mask, nullptr));
  return GF_OK;
}

gf_status gf_convolve_psf(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *in, int n_ch, float *out) {
  ProfBind pb_(c);
  if (!c || !b || !p || !in || !out) return fail(c, GF_EINVAL, "gf_convolve_psf: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_convolve_psf: PSF prepared for another batch");
  if (n_ch < 1 || n_ch > 64) return fail(c, GF_EINVAL, "gf_convolve_psf: n_ch out of range");
  Arena a;
  a.take<float2>(p->n_s1 * n_ch);
  a.take<float2>(p->n_s2 * n_ch);
  gf_status st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  float2 *S1 = a.take<float2>(p->n_s1 * n_ch);
  float2 *S2 = a.take<float2>(p->n_s2 * n_ch);
  return convolve(c, b, p, in, n_ch, out, S1, S2, nullptr);
}

gf_status gf_chi2(gf_ctx *c, const gf_batch *b, const float *model, const float *theta, const float *data,
                  const float *weight, float *resid, float *chi2) {
  ProfBind pb_(c);
  if (!c || !b || !model || !theta || !data || !weight || !chi2) return fail(c, GF_EINVAL, "gf_chi2: null argument");
  gf_status st = ensure_counters(c, b->n);
  if (st != GF_OK) return st;
  Arena a;
  a.take<float2>((int64_t)b->h_pix.size());
  st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  float2 *part = a.take<float2>((int64_t)b->h_pix.size());
  GF_TRY(c, launch_chi2(c->stream, b, model, theta, false, data, weight, resid, part, c->d_counters,
                        (float2 *)chi2, nullptr));
  return GF_OK;
}

static void likelihood_layout(const gf_batch *b, const gf_psf *p, Arena &a, float **mpad, float **mconv,
                              float2 **S1, float2 **S2, float2 **part) {
  *mpad = a.take<float>(b->n_pad);
  *mconv = a.take<float>(b->n_pix);
  *S1 = a.take<float2>(p->n_s1);
  *S2 = a.take<float2>(p->n_s2);
  *part = a.take<float2>(chi2_slots(b, p));
}

int64_t gf_likelihood_workspace(const gf_batch *b, const gf_psf *p) {
  if (!b || !p) return -1;
  Arena a;
  float *m1, *m2;
  float2 *s1, *s2, *pt;
  likelihood_layout(b, p, a, &m1, &m2, &s1, &s2, &pt);
  return (int64_t)a.off;
}

gf_status gf_likelihood(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *theta, int S, const float *data,
                        const float *weight, float *chi2, void *work) {
  ProfBind pb_(c);
  if (!c || !b || !p || !theta || !data || !weight || !chi2) return fail(c, GF_EINVAL, "gf_likelihood: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_likelihood: PSF prepared for another batch");
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return fail(c, GF_EINVAL, "gf_likelihood: oversample out of range");
  gf_status st = ensure_counters(c, b->n);
  if (st != GF_OK) return st;
  if (!work) {
    st = ensure_ws(c, (size_t)gf_likelihood_workspace(b, p));
    if (st != GF_OK) return st;
    work = c->ws;
  }
  Arena a{(char *)work, 0};
  float *mpad, *mconv;
  float2 *S1, *S2, *part;
  likelihood_layout(b, p, a, &mpad, &mconv, &S1, &S2, &part);
  GF_TRY(c, launch_eval(c->stream, b, theta, S, c->d_bn, mpad, nullptr));
  GF_TRY(c, conv_chi2(c->stream, b, p, mpad, S1, S2, mconv, theta, false, data, weight, part, nullptr, nullptr, &c->fork));
  GF_TRY(c, launch_pair_final(c->stream, b->n, p->d_c2_first, part, (float2 *)chi2, nullptr));
  return GF_OK;
}

gf_status gf_model(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *theta, int S, float *out,
                   void *work) {
  ProfBind pb_(c);
  if (!c || !b || !p || !theta || !out) return fail(c, GF_EINVAL, "gf_model: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_model: PSF prepared for another batch");
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return fail(c, GF_EINVAL, "gf_model: oversample out of range");
  if (!work) {
    gf_status st = ensure_ws(c, (size_t)gf_likelihood_workspace(b, p));
    if (st != GF_OK) return st;
    work = c->ws;
  }
  Arena a{(char *)work, 0};
  float *mpad, *mconv;
  float2 *S1, *S2, *part;
  likelihood_layout(b, p, a, &mpad, &mconv, &S1, &S2, &part);
  GF_TRY(c, launch_eval(c->stream, b, theta, S, c->d_bn, mpad, nullptr));
  gf_status st = convolve(c, b, p, mpad, 1, out, S1, S2, nullptr);
  if (st != GF_OK) return st;
  GF_TRY(c, launch_add_sky(c->stream, b, theta, out));
  return GF_OK;
}

// -------------------------------------------------------------- derivatives
gf_status gf_jacobian(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *theta, int S, int mode,
                      const float *cot, const float *weight, float scale, float *out) {
  ProfBind pb_(c);
  if (!c || !b || !p || !theta || !out) return fail(c, GF_EINVAL, "gf_jacobian: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_jacobian: PSF prepared for another batch");
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return fail(c, GF_EINVAL, "gf_jacobian: oversample out of range");
  if (mode == GF_JAC_FULL) {
    const int nchan = kNPC * b->max_nc;
    Arena a;
    a.take<float>(b->n_pad * nchan);
    a.take<float>(b->n_pix * nchan);
    a.take<float2>(p->n_s1 * nchan);
    a.take<float2>(p->n_s2 * nchan);
    gf_status st = ensure_ws(c, a.off);
    if (st != GF_OK) return st;
    a = Arena{(char *)c->ws, 0};
    float *cpad = a.take<float>(b->n_pad * nchan);
    float *jc = a.take<float>(b->n_pix * nchan);
    float2 *S1 = a.take<float2>(p->n_s1 * nchan);
    float2 *S2 = a.take<float2>(p->n_s2 * nchan);
    GF_TRY(c, launch_eval_jac(c->stream, b, theta, S, c->d_bn, cpad, nchan, nullptr));
    st = convolve(c, b, p, cpad, nchan, jc, S1, S2, nullptr);
    if (st != GF_OK) return st;
    GF_TRY(c, launch_jac_assemble(c->stream, b, jc, nchan, out));
    return GF_OK;
  }
  if (mode != GF_JAC_ADJOINT) return fail(c, GF_EINVAL, "gf_jacobian: unknown mode");
  if (!cot) return fail(c, GF_EINVAL, "gf_jacobian: adjoint mode needs a cotangent image");
  Arena a;
  a.take<float>(b->n_pix);
  a.take<float2>((int64_t)b->h_pix.size());
  a.take<float2>(p->n_s1a);
  a.take<float2>(p->n_s2a);
  a.take<float>(b->n_pad);
  a.take<float>((int64_t)b->h_eval.size() * (kMaxP - 1));
  gf_status st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  float *cimg = a.take<float>(b->n_pix);
  float2 *spart = a.take<float2>((int64_t)b->h_pix.size());
  float2 *S1 = a.take<float2>(p->n_s1a);
  float2 *S2 = a.take<float2>(p->n_s2a);
  float *adj = a.take<float>(b->n_pad);
  float *cpart = a.take<float>((int64_t)b->h_eval.size() * (kMaxP - 1));
  GF_TRY(c, launch_cot_prep(c->stream, b, cot, weight, scale, cimg, spart));
  GF_TRY(c, launch_fft_corr(c->stream, b, p, cimg, S1, S2, adj));
  GF_TRY(c, launch_direct(c->stream, b, p, cimg, 1, adj, true, nullptr, nullptr));
  GF_TRY(c, launch_adjoint_contract(c->stream, b, theta, S, c->d_bn, adj, cpart));
  GF_TRY(c, launch_adjoint_final(c->stream, b, b->d_eval_first, cpart, spart, out));
  return GF_OK;
}

// ------------------------------------------------------------------ LM fit
void gf_lm_opts_default(gf_lm_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(gf_lm_opts);
  o->max_iter = 100;
  o->oversample = 5;
  o->lambda0 = 1e-3;
  o->lambda_up = 10.0;
  o->lambda_down = 10.0;
  o->lambda_max = 1e10;
  o->ftol = 1e-5;
  o->xtol = 1e-10;
  o->lo = nullptr;
  o->hi = nullptr;
  o->free_mask = nullptr;
  o->poll_every = 4;
  o->use_graph = 1;
  o->speculate = -1;
  o->start = nullptr;
}

namespace {

struct LMBufs {
  float *cpad, *jc, *mpad, *mconv, *npart;
  // Spectra of the multi-pass FFT: S1/S2 for the Jacobian images (nchan
  // channels a stamp), S1c/S2c for the one-channel chi^2 convolutions.  A
  // stamp's block starts at its offset times the channel count, so the two
  // layouts overlap across stamps: they get separate buffers because the two
  // lanes run one's chi^2 pass while the other convolves its Jacobians.
  float2 *S1, *S2, *S1c, *S2c, *cpart;
  float2 *gpart;   // chi^2 partials per normal-equation unit (speculative iterations)
  double *Ag, *theta_t;
  LMState *st;
  int *mjac, *mtrial, *cnt;
  Work *lists;   // compacted work lists of the stamps still iterating
  CopyRun *plan;   // the copies that restrict them
  CompC *cc_th, *cc_t;   // component constants of theta and of the trial point
};

int64_t full_list_units(const gf_batch *b, const gf_psf *p) {
  return (int64_t)b->h_eval.size() + b->h_pix.size() + b->h_neq.size() + p->h_rows.size() + p->h_cols.size() +
         p->h_irows.size() + p->h_rows_n.size() + p->h_cols_n.size() + p->h_irows_n.size() + p->h_direct.size() +
         p->h_pix_direct.size() + p->h_f2d.size() + p->h_rows_alt.size() + p->h_cols_alt.size() +
         p->h_irows_alt.size() + p->h_rows_n_alt.size() + p->h_cols_n_alt.size() + p->h_irows_n_alt.size() + b->n;
}

// The lists an LM fit restricts, in a fixed order: the batch's evaluation,
// chi^2 and Gram units, the PSF's multi-pass units (both launch shapes),
// direct tiles and chi^2 units, one-workgroup entries, and the multi-pass
// units kept for the one-workgroup stamps.
enum {
  RL_EVAL, RL_PIX, RL_NEQ, RL_ROWS, RL_COLS, RL_IROWS, RL_ROWS_N, RL_COLS_N, RL_IROWS_N, RL_DIRECT, RL_PIX_DIRECT,
  RL_F2D, RL_ROWS_ALT, RL_COLS_ALT, RL_IROWS_ALT, RL_ROWS_N_ALT, RL_COLS_N_ALT, RL_IROWS_N_ALT, RL_COUNT
};

static void lm_lists(const gf_batch *b, const gf_psf *p, const std::vector<Work> *h[RL_COUNT],
                     const Work *d[RL_COUNT]) {
  const std::vector<Work> *hh[RL_COUNT] = {&b->h_eval, &b->h_pix, &b->h_neq, &p->h_rows, &p->h_cols, &p->h_irows,
                                           &p->h_rows_n, &p->h_cols_n, &p->h_irows_n, &p->h_direct,
                                           &p->h_pix_direct, &p->h_f2d, &p->h_rows_alt, &p->h_cols_alt,
                                           &p->h_irows_alt, &p->h_rows_n_alt, &p->h_cols_n_alt, &p->h_irows_n_alt};
  const Work *dd[RL_COUNT] = {b->d_eval, b->d_pix, b->d_neq, p->d_rows, p->d_cols, p->d_irows, p->d_rows_n,
                              p->d_cols_n, p->d_irows_n, p->d_direct, p->d_pix_direct, p->d_f2d, p->d_rows_alt,
                              p->d_cols_alt, p->d_irows_alt, p->d_rows_n_alt, p->d_cols_n_alt, p->d_irows_n_alt};
  for (int k = 0; k < RL_COUNT; ++k) {
    h[k] = hh[k];
    d[k] = dd[k];
  }
}

// Runs of every restricted list (built once per PSF); returns their total.
static int64_t lm_runs_ensure(const gf_batch *b, const gf_psf *p) {
  if (p->lm_runs.empty()) {
    const std::vector<Work> *h[RL_COUNT];
    const Work *d[RL_COUNT];
    lm_lists(b, p, h, d);
    p->lm_runs.resize(RL_COUNT);
    for (int k = 0; k < RL_COUNT; ++k) {
      ListRuns &r = p->lm_runs[k];
      const std::vector<Work> &v = *h[k];
      for (size_t i = 0; i < v.size(); ++i) {
        if (i == 0 || v[i].stamp != v[i - 1].stamp) {
          r.stamp.push_back(v[i].stamp);
          r.beg.push_back((int32_t)i);
          r.len.push_back(0);
        }
        ++r.len.back();
      }
    }
  }
  int64_t n = 0;
  for (const ListRuns &r : p->lm_runs) n += (int64_t)r.stamp.size();
  return n;
}

// Work lists restricted to the stamps flagged in act, taken run by run from
// the full device lists into dev (one copy launch over a plan uploaded to
// plan_dev); the view points into dev.  Stamps of a one-workgroup bucket
// with fewer active stamps than the context's minimum are flagged in moved
// and take their multi-pass units from then on (the flag stays set for the
// rest of the fit).  Each list keeps the order of the full list, followed
// for the multi-pass lists by the moved stamps' units.
hipError_t restrict_lists(hipStream_t st, const gf_batch *b, const gf_psf *p, const std::vector<char> &act,
                          std::vector<char> &moved, CopyRun *plan_dev, Work *dev, WorkView &v) {
  const std::vector<Work> *h[RL_COUNT];
  const Work *d[RL_COUNT];
  lm_lists(b, p, h, d);
  const std::vector<ListRuns> &R = p->lm_runs;
  // buckets with few stamps left would not fill the device: their stamps
  // move to the multi-pass launches, which spread a stamp over many
  // workgroups
  {
    const ListRuns &rf = R[RL_F2D];
    int cnt[kF2dBuckets] = {};
    for (size_t i = 0; i < rf.stamp.size(); ++i)
      if (act[rf.stamp[i]] && !moved[rf.stamp[i]]) ++cnt[(*h[RL_F2D])[rf.beg[i]].unit];
    for (size_t i = 0; i < rf.stamp.size(); ++i) {
      const int s = rf.stamp[i];
      if (act[s] && !moved[s] && cnt[(*h[RL_F2D])[rf.beg[i]].unit] < b->ctx->f2d_min_active[(*h[RL_F2D])[rf.beg[i]].unit])
        moved[s] = 1;
    }
  }
  std::vector<CopyRun> plan;
  int64_t off = 0;
  // which: 0 every active stamp, 1 active stamps not moved, 2 active moved stamps
  auto take = [&](int k, int which) {
    const ListRuns &r = R[k];
    for (size_t i = 0; i < r.stamp.size(); ++i) {
      const int s = r.stamp[i];
      if (!act[s] || (which == 1 && moved[s]) || (which == 2 && !moved[s])) continue;
      plan.push_back(CopyRun{d[k] + r.beg[i], off, r.len[i], 0});
      off += r.len[i];
    }
  };
  auto put = [&](int k, int alt, const Work *&ptr, int &n) {
    const int64_t start = off;
    take(k, k == RL_F2D ? 1 : 0);
    if (alt >= 0) take(alt, 2);
    ptr = dev + start;
    n = (int)(off - start);
  };
  put(RL_EVAL, -1, v.eval, v.n_eval);
  put(RL_PIX, -1, v.pix, v.n_pix);
  put(RL_NEQ, -1, v.neq, v.n_neq);
  put(RL_ROWS, RL_ROWS_ALT, v.rows, v.n_rows);
  put(RL_COLS, RL_COLS_ALT, v.cols, v.n_cols);
  put(RL_IROWS, RL_IROWS_ALT, v.irows, v.n_irows);
  put(RL_ROWS_N, RL_ROWS_N_ALT, v.rows_n, v.n_rows_n);
  put(RL_COLS_N, RL_COLS_N_ALT, v.cols_n, v.n_cols_n);
  put(RL_IROWS_N, RL_IROWS_N_ALT, v.irows_n, v.n_irows_n);
  put(RL_DIRECT, -1, v.direct, v.n_direct);
  put(RL_PIX_DIRECT, -1, v.pix_direct, v.n_pix_direct);
  int n_f2d = 0;
  put(RL_F2D, -1, v.f2d, n_f2d);
  // the units of stamps >= kNeqBigPix lead the Gram list, as in the full list
  v.n_neq_big = 0;
  {
    const ListRuns &r = R[RL_NEQ];
    for (size_t i = 0; i < r.stamp.size(); ++i)
      if (act[r.stamp[i]] && b->h_desc[r.stamp[i]].H * b->h_desc[r.stamp[i]].W >= kNeqBigPix) v.n_neq_big += r.len[i];
  }
  for (int k = 0; k <= kF2dBuckets; ++k) v.f2d_first[k] = 0;
  {
    const ListRuns &r = R[RL_F2D];
    for (size_t i = 0; i < r.stamp.size(); ++i)
      if (act[r.stamp[i]] && !moved[r.stamp[i]]) ++v.f2d_first[(*h[RL_F2D])[r.beg[i]].unit + 1];
  }
  for (int k = 0; k < kF2dBuckets; ++k) v.f2d_first[k + 1] += v.f2d_first[k];
  // the per-stamp LM kernels' list: the active stamps, from the host
  std::vector<Work> stamps;
  for (int s = 0; s < b->n; ++s)
    if (act[s]) stamps.push_back({s, 0});
  v.stamps = dev + off;
  v.n_stamps = (int)stamps.size();
  hipError_t e = hipSuccess;
  if (!stamps.empty())
    e = hipMemcpyAsync(dev + off, stamps.data(), stamps.size() * sizeof(Work), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !plan.empty())
    e = hipMemcpyAsync(plan_dev, plan.data(), plan.size() * sizeof(CopyRun), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_copy_runs(st, plan_dev, (int)plan.size(), dev);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors must outlive the copies
  return e;
}

void lm_layout(const gf_batch *b, const gf_psf *p, int nchan, int nacc, Arena &a, LMBufs &B) {
  B.cpad = a.take<float>(b->n_pad * nchan);
  B.jc = a.take<float>(b->n_pix * nchan);
  B.S1 = a.take<float2>(p->n_s1 * nchan);
  B.S2 = a.take<float2>(p->n_s2 * nchan);
  B.S1c = a.take<float2>(p->n_s1);
  B.S2c = a.take<float2>(p->n_s2);
  B.npart = a.take<float>((int64_t)b->h_neq.size() * nacc);
  B.Ag = a.take<double>((int64_t)b->n * (kMaxP * kMaxP + kMaxP));
  B.theta_t = a.take<double>(b->n_par);
  B.mpad = a.take<float>(b->n_pad);
  B.mconv = a.take<float>(b->n_pix);
  B.cpart = a.take<float2>(chi2_slots(b, p));
  B.gpart = a.take<float2>((int64_t)b->h_neq.size());
  B.st = a.take<LMState>(b->n);
  B.mjac = a.take<int>(b->n);
  B.mtrial = a.take<int>(b->n);
  B.cnt = a.take<int>(8 * std::max(2, kLmLanes));
  // room for the lists and copy plans of every lane (each up to the full size)
  B.lists = a.take<Work>(std::max(2, kLmLanes) * full_list_units(b, p));
  B.plan = a.take<CopyRun>(std::max(2, kLmLanes) * (lm_runs_ensure(b, p) + 1));
  B.cc_th = a.take<CompC>((int64_t)b->n * kMaxComp);
  B.cc_t = a.take<CompC>((int64_t)b->n * kMaxComp);
}

}  // namespace

gf_status gf_fit_lm(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *data, const float *weight,
                    double *theta, const gf_lm_opts *opts, gf_lm_result *res) {
  ProfBind pb_(c);
  if (!c || !b || !p || !data || !weight || !theta || !res) return fail(c, GF_EINVAL, "gf_fit_lm: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_fit_lm: PSF prepared for another batch");
  if (opts && opts->struct_size != (int32_t)sizeof(gf_lm_opts))
    return fail(c, GF_EINVAL, "gf_fit_lm: opts->struct_size differs from sizeof(gf_lm_opts) (initialise with gf_lm_opts_default)");
  gf_lm_opts o;
  if (opts) o = *opts; else gf_lm_opts_default(&o);
  if (o.max_iter < 0 || o.oversample < 1 || o.oversample > GF_MAX_OVERSAMPLE || !(o.lambda_up > 1.0) ||
      !(o.lambda_down > 1.0) || !(o.lambda0 > 0.0) || o.speculate < -1 || o.speculate > 1)
    return fail(c, GF_EINVAL, "gf_fit_lm: invalid options");
  const bool spec = o.speculate > 0 || (o.speculate < 0 && b->n == 1);
  if (o.poll_every < 1) o.poll_every = 1;
  if (o.start == theta) o.start = nullptr;
  if (b->max_nc > 2) return fail(c, GF_ESHAPE, "gf_fit_lm: at most two components per stamp");
  const int nchan = kNPC * b->max_nc;
  const int nacc = 256;  // 16 x 16 Gram matrix per workgroup
  gf_status st = ensure_counters(c, b->n);
  if (st != GF_OK) return st;
  Arena a;
  LMBufs B;
  lm_layout(b, p, nchan, nacc, a, B);
  st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  lm_layout(b, p, nchan, nacc, a, B);
  const size_t states_bytes = (size_t)b->n * sizeof(LMState);
  if (b->n > 1 && c->h_states_bytes < states_bytes) {   // no copy into it is in flight between fits
    if (c->h_states) (void)hipHostFree(c->h_states);
    c->h_states = nullptr;
    c->h_states_bytes = 0;
    if (hipHostMalloc(&c->h_states, states_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(c, GF_ENOMEM, "gf_fit_lm: pinned host memory for the LM states");
    c->h_states_bytes = states_bytes;
  }
  const int S = o.oversample;

  // The fit runs on the context's LM stream, joined to the caller's stream
  // by an event at both ends.  The captured iteration over the full work
  // lists stays in the context and is replayed by later calls with the same
  // key; graphs over compacted lists belong to this call only.
  if (!c->lm_stream) GF_TRY(c, hipStreamCreateWithFlags(&c->lm_stream, hipStreamNonBlocking));
  if (!c->lm_ev) GF_TRY(c, hipEventCreateWithFlags(&c->lm_ev, hipEventDisableTiming));
  hipStream_t cs = c->lm_stream;
  hipEvent_t ev = c->lm_ev;
  LmGraphKey key;
  key.batch_uid = b->uid;
  key.psf_uid = p->uid;
  key.data = data;
  key.weight = weight;
  key.theta = theta;
  key.ws = c->ws;
  key.lo = o.lo;
  key.hi = o.hi;
  key.free_mask = o.free_mask;
  key.max_iter = o.max_iter;
  key.oversample = o.oversample;
  key.spec = spec ? 1 : 0;
  key.lambda_up = o.lambda_up;
  key.lambda_down = o.lambda_down;
  key.lambda_max = o.lambda_max;
  key.ftol = o.ftol;
  key.xtol = o.xtol;
  const bool graphs = o.use_graph && o.max_iter > 0;
  const bool reuse = graphs && c->lm_exec && c->lm_key == key;
  if (graphs && !reuse && c->lm_exec) {
    // nothing of an earlier call may still be replaying the graph
    GF_TRY(c, hipStreamSynchronize(cs));
    (void)hipGraphExecDestroy(c->lm_exec);
    (void)hipGraphDestroy(c->lm_graph);
    c->lm_exec = nullptr;
    c->lm_graph = nullptr;
    c->lm_key = LmGraphKey{};
  }
  // batches of at least this many stamps run their plain-form iterations in
  // two lanes (see run below)
  constexpr int kLmLaneMin = 512;
  const int lanes = (!spec && graphs && b->n >= kLmLaneMin) ? kLmLanes : 1;
  if (lanes > 1) {
    for (hipStream_t &s : c->lm_lane_stream)
      if (!s) GF_TRY(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (hipEvent_t &e : c->lm_lane_ev)
      if (!e) GF_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  hipGraph_t vgraph = nullptr;
  hipGraphExec_t vexec = nullptr;
  hipGraphExec_t exec = reuse ? c->lm_exec : nullptr;
  auto cleanup = [&]() {
    if (vexec) (void)hipGraphExecDestroy(vexec);
    if (vgraph) (void)hipGraphDestroy(vgraph);
  };
  auto run = [&]() -> gf_status {
    GF_TRY(c, hipEventRecord(ev, c->stream));
    GF_TRY(c, hipStreamWaitEvent(cs, ev, 0));
    // start point: clip and set up, evaluate, chi2 (speculative: the Jacobian images and
    // normal equations of the start point, chi^2 from the same model)
    GF_TRY(c, launch_lm_start(cs, b, o.start, theta, o.lo, o.hi, B.theta_t, S, c->d_bn, B.cc_th));
    if (spec) {
      GF_TRY(c, launch_eval_jac_d(cs, b, B.theta_t, S, c->d_bn, B.cpad, nchan, nullptr, nullptr, B.cc_th, false));
      GF_TRY(c, launch_fft_conv(cs, b, p, B.cpad, nchan, B.S1, B.S2, B.jc, nullptr, nullptr, nullptr, &c->fork));
      GF_TRY(c, launch_direct(cs, b, p, B.cpad, nchan, B.jc, false, nullptr, nullptr));
      GF_TRY(c, launch_normal_eq(cs, b, B.jc, B.theta_t, data, weight, B.npart, nacc, nchan, nullptr, nullptr,
                                 B.gpart));
      GF_TRY(c, launch_lm_init(cs, b, o.lambda0, b->d_neq_first, B.gpart, B.st, B.mjac, B.mtrial, B.cnt));
    } else {
      GF_TRY(c, launch_eval_d(cs, b, B.theta_t, S, c->d_bn, B.mpad, nullptr, nullptr, B.cc_th, false));
      GF_TRY(c, conv_chi2(cs, b, p, B.mpad, B.S1c, B.S2c, B.mconv, B.theta_t, true, data, weight, B.cpart, nullptr,
                          nullptr, &c->fork, true));
      GF_TRY(c, launch_lm_init(cs, b, o.lambda0, p->d_c2_first, B.cpart, B.st, B.mjac, B.mtrial, B.cnt, 1));
    }
    WorkView view;
    const WorkView *vw = nullptr;   // null: the full lists
    std::vector<char> moved(b->n, 0);   // one-workgroup stamps moved to the multi-pass launches
    int view_stamps = b->n;
    // Speculative iteration: solve, then Jacobian images, normal equations
    // and chi^2 at the trial point, accept or reject.  An accepted trial
    // leaves its normal equations for the next solve; after a rejection the
    // solve reuses the stored system of the current point.
    // the stream, lists and active count the iteration below launches on:
    // the fit's stream and lists, or one lane's (see run_lanes)
    hipStream_t xs = cs;
    int *xcnt = B.cnt;
    auto iteration_spec = [&]() -> gf_status {
      GF_TRY(c, launch_lm_solve(xs, b, B.npart, &o, B.st, B.Ag, theta, B.theta_t, B.mjac, B.mtrial, xcnt, B.cc_th,
                                B.cc_t, c->d_bn, vw));
      GF_TRY(c, launch_eval_jac_d(xs, b, B.theta_t, S, c->d_bn, B.cpad, nchan, B.mtrial, vw, B.cc_t, false));
      GF_TRY(c, launch_fft_conv(xs, b, p, B.cpad, nchan, B.S1, B.S2, B.jc, B.mtrial, vw, nullptr, &c->fork));
      GF_TRY(c, launch_direct(xs, b, p, B.cpad, nchan, B.jc, false, B.mtrial, vw));
      GF_TRY(c, launch_normal_eq(xs, b, B.jc, B.theta_t, data, weight, B.npart, nacc, nchan, B.mtrial, vw,
                                 B.gpart));
      GF_TRY(c, launch_lm_update(xs, b, &o, b->d_neq_first, B.gpart, B.st, theta, B.theta_t, B.mjac, B.mtrial,
                                 xcnt, B.cc_th, B.cc_t, vw));
      return GF_OK;
    };
    auto iteration = [&]() -> gf_status {
      if (spec) return iteration_spec();
      GF_TRY(c, launch_eval_jac_d(xs, b, theta, S, c->d_bn, B.cpad, nchan, B.mjac, vw, B.cc_th, false));
      GF_TRY(c, launch_fft_conv(xs, b, p, B.cpad, nchan, B.S1, B.S2, B.jc, B.mjac, vw, nullptr, &c->fork));
      GF_TRY(c, launch_direct(xs, b, p, B.cpad, nchan, B.jc, false, B.mjac, vw));
      GF_TRY(c, launch_normal_eq(xs, b, B.jc, theta, data, weight, B.npart, nacc, nchan, B.mjac, vw, nullptr, 0,
                                 B.mconv));
      GF_TRY(c, launch_lm_solve(xs, b, B.npart, &o, B.st, B.Ag, theta, B.theta_t, B.mjac, B.mtrial, xcnt, B.cc_th,
                                B.cc_t, c->d_bn, vw));
      GF_TRY(c, launch_eval_d(xs, b, B.theta_t, S, c->d_bn, B.mpad, B.mtrial, vw, B.cc_t, false));
      GF_TRY(c, conv_chi2(xs, b, p, B.mpad, B.S1c, B.S2c, B.mconv, B.theta_t, true, data, weight, B.cpart, B.mtrial,
                          vw, &c->fork, true));
      GF_TRY(c, launch_lm_update(xs, b, &o, p->d_c2_first, B.cpart, B.st, theta, B.theta_t, B.mjac, B.mtrial,
                                 xcnt, B.cc_th, B.cc_t, vw, 1));
      return GF_OK;
    };
    // capture one iteration into (g, e), replacing what they held
    auto capture = [&](hipGraph_t &g, hipGraphExec_t &e) -> gf_status {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      e = nullptr;
      g = nullptr;
      GF_TRY(c, hipStreamBeginCapture(xs, hipStreamCaptureModeThreadLocal));
      gf_status s2 = iteration();
      hipError_t ce = hipStreamEndCapture(xs, &g);
      if (s2 != GF_OK) return s2;
      GF_TRY(c, ce);
      GF_TRY(c, hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
      return GF_OK;
    };
    // Two lanes: a large plain-form batch runs as two halves (the stamps of
    // even and of odd index), each with its own work lists, active count,
    // iteration graph and restrictions, on two streams, so the tail of one
    // half's launches overlaps the other half's work.  A stamp runs the same
    // kernels as in one lane; only the moves of one-workgroup stamps to the
    // multi-pass launches follow its half's counts.  Results are written once
    // both halves have finished.
    if (lanes > 1) {
      struct Lane {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        WorkView view;
        int stamps = 0;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        int *cnt = nullptr;
        Work *dev = nullptr;
        CopyRun *plan = nullptr;
        volatile int *h = nullptr;
        bool done = false;
      };
      Lane ln[kLmLanes];
      // After a normal end every replay has been waited for at a poll; after
      // an error, replays may still run, so the lanes' streams are waited
      // for before their graphs go.
      auto lanes_cleanup = [&](bool failed) {
        for (Lane &l : ln)
          if (failed && l.s) (void)hipStreamSynchronize(l.s);
        for (Lane &l : ln) {
          if (l.x) (void)hipGraphExecDestroy(l.x);
          if (l.g) (void)hipGraphDestroy(l.g);
          l.x = nullptr;
          l.g = nullptr;
        }
      };
      auto body = [&]() -> gf_status {
        const int64_t units = full_list_units(b, p), runs = lm_runs_ensure(b, p) + 1;
        for (int l = 0; l < kLmLanes; ++l) {
          ln[l].s = l == 0 ? cs : c->lm_lane_stream[l - 1];
          ln[l].e = c->lm_lane_ev[l];
          ln[l].cnt = B.cnt + 8 * l;
          ln[l].dev = B.lists + units * l;
          ln[l].plan = B.plan + runs * l;
          ln[l].h = c->h_pinned + 8 * l;
        }
        std::vector<char> half(b->n);
        for (int l = 0; l < kLmLanes; ++l) {   // the lanes' lists (the start point is done on cs)
          for (int q = 0; q < b->n; ++q) half[q] = q % kLmLanes == l;
          GF_TRY(c, restrict_lists(cs, b, p, half, moved, ln[l].plan, ln[l].dev, ln[l].view));
          ln[l].stamps = ln[l].view.n_stamps;
        }
        GF_TRY(c, hipEventRecord(ln[0].e, cs));
        for (int l = 1; l < kLmLanes; ++l) GF_TRY(c, hipStreamWaitEvent(ln[l].s, ln[0].e, 0));
        auto use = [&](Lane &l) {
          xs = l.s;
          vw = &l.view;
          xcnt = l.cnt;
        };
        // Each lane runs poll_every iterations, then its count is copied; the
        // host waits on the lanes' polls in turn, so while it waits on (and
        // restricts) one lane the other's queued iterations keep the device
        // busy.
        int itl[kLmLanes] = {};
        bool pending[kLmLanes] = {};
        int next = 0;
        for (;;) {
          for (int li = 0; li < kLmLanes; ++li) {
            Lane &l = ln[li];
            if (l.done || pending[li]) continue;
            use(l);
            do {
              if (l.x && itl[li] > 0) {
                GF_TRY(c, hipGraphLaunch(l.x, l.s));
              } else {
                gf_status s2 = iteration();
                if (s2 != GF_OK) return s2;
              }
              if (itl[li] == 0 && o.max_iter > 1) {
                gf_status s2 = capture(l.g, l.x);
                if (s2 != GF_OK) return s2;
              }
              ++itl[li];
            } while (itl[li] % o.poll_every != 0 && itl[li] < o.max_iter);
            GF_TRY(c, hipMemcpyAsync((void *)l.h, l.cnt, sizeof(int), hipMemcpyDeviceToHost, l.s));
            GF_TRY(c, hipEventRecord(l.e, l.s));
            pending[li] = true;
          }
          int li = next;
          for (int k = 0; k < kLmLanes && !pending[li]; ++k) li = (li + 1) % kLmLanes;
          if (!pending[li]) break;   // every lane done
          next = (li + 1) % kLmLanes;
          Lane &l = ln[li];
          GF_TRY(c, hipEventSynchronize(l.e));
          pending[li] = false;
          const int active = *l.h;
          if (active == 0 || itl[li] >= o.max_iter) {
            l.done = true;
            continue;
          }
          if (2 * active <= l.stamps) {
            GF_TRY(c, hipMemcpyAsync(c->h_states, B.st, b->n * sizeof(LMState), hipMemcpyDeviceToHost, l.s));
            GF_TRY(c, hipStreamSynchronize(l.s));
            const LMState *hs = static_cast<const LMState *>(c->h_states);
            for (int q = 0; q < b->n; ++q) half[q] = (q % kLmLanes == li && hs[q].active) ? 1 : 0;
            GF_TRY(c, restrict_lists(l.s, b, p, half, moved, l.plan, l.dev, l.view));
            l.stamps = active;
            use(l);
            gf_status s2 = capture(l.g, l.x);
            if (s2 != GF_OK) return s2;
          }
        }
        // both halves joined on the fit's stream, then every stamp's result
        for (int l = 1; l < kLmLanes; ++l) {
          GF_TRY(c, hipEventRecord(ln[l].e, ln[l].s));
          GF_TRY(c, hipStreamWaitEvent(cs, ln[l].e, 0));
        }
        GF_TRY(c, launch_lm_result(cs, b->n, B.st, res));
        GF_TRY(c, hipEventRecord(ev, cs));
        GF_TRY(c, hipStreamWaitEvent(c->stream, ev, 0));
        return GF_OK;
      };
      const gf_status s2 = body();
      lanes_cleanup(s2 != GF_OK);
      return s2;
    }
    std::vector<char> act;
    // the result records are written before every poll, so a fit that the
    // poll finds finished returns without another launch; the host waits
    // only for the count
    bool res_fresh = false;
    for (int it = 0; it < o.max_iter; ++it) {
      // The first iteration is launched kernel by kernel, so the device starts
      // on it while the host is still enqueueing (a graph launch hands over
      // nothing until the whole graph is submitted); the graph, captured here
      // when the context holds none for this key, replays the rest.
      if (exec && it > 0) {
        GF_TRY(c, hipGraphLaunch(exec, cs));
      } else {
        gf_status s2 = iteration();
        if (s2 != GF_OK) return s2;
      }
      if (it == 0 && graphs && !reuse && o.max_iter > 1) {
        gf_status s2 = capture(c->lm_graph, c->lm_exec);
        if (s2 != GF_OK) return s2;
        c->lm_key = key;
        exec = c->lm_exec;
      }
      res_fresh = false;
      if ((it + 1) % o.poll_every == 0 || it + 1 == o.max_iter) {
        GF_TRY(c, hipMemcpyAsync(c->h_pinned, B.cnt, sizeof(int), hipMemcpyDeviceToHost, cs));
        GF_TRY(c, hipEventRecord(ev, cs));
        GF_TRY(c, launch_lm_result(cs, b->n, B.st, res));
        res_fresh = true;
        GF_TRY(c, hipEventSynchronize(ev));
        const int active = *(volatile int *)c->h_pinned;
        if (active == 0) break;
        // Once half of the stamps in the current lists have finished, restrict
        // the lists to the stamps still iterating (finished stamps would
        // otherwise still cost their workgroups in every launch).
        if (b->n > 1 && 2 * active <= view_stamps && it + 1 < o.max_iter) {
          // on the fit's stream (not the legacy stream, which would wait
          // for other host threads' streams, possibly capturing)
          GF_TRY(c, hipMemcpyAsync(c->h_states, B.st, b->n * sizeof(LMState), hipMemcpyDeviceToHost, cs));
          GF_TRY(c, hipStreamSynchronize(cs));
          const LMState *hs = static_cast<const LMState *>(c->h_states);
          act.assign(b->n, 0);
          for (int q = 0; q < b->n; ++q) act[q] = hs[q].active ? 1 : 0;
          GF_TRY(c, restrict_lists(cs, b, p, act, moved, B.plan, B.lists, view));
          vw = &view;
          view_stamps = active;
          if (exec) {
            gf_status s2 = capture(vgraph, vexec);
            if (s2 != GF_OK) return s2;
            exec = vexec;
          }
        }
      }
    }
    if (!res_fresh) GF_TRY(c, launch_lm_result(cs, b->n, B.st, res));
    GF_TRY(c, hipEventRecord(ev, cs));
    GF_TRY(c, hipStreamWaitEvent(c->stream, ev, 0));
    return GF_OK;
  };
  st = run();
  if (st != GF_OK) (void)hipStreamSynchronize(cs);   // replays of this call's graph may still run
  cleanup();
  return st;
}

gf_status gf_group_best(gf_ctx *c, const gf_batch *b, const gf_lm_result *res, const double *theta, double *best,
                        int32_t *best_stamp) {
  if (!c || !b || !res || !theta || !best) return fail(c, GF_EINVAL, "gf_group_best: null argument");
  ProfBind pb_(c);
  GF_TRY(c, launch_group_best(c->stream, b, res, theta, best, best_stamp));
  return GF_OK;
}

int gf_batch_groups(const gf_batch *b) { return b ? b->n_groups : 0; }

gf_status gf_expand_starts(gf_ctx *c, int n_groups, int n_starts, const double *theta0, double *out) {
  if (!c || n_groups < 0 || n_starts < 1 || n_starts > 4 || (n_groups > 0 && (!theta0 || !out)))
    return fail(c, GF_EINVAL, "gf_expand_starts: bad argument (1 <= n_starts <= 4)");
  GF_TRY(c, launch_expand_starts(c->stream, n_groups, n_starts, theta0, out));
  return GF_OK;
}

// ---------------------------------------------------------------- simplex
void gf_simplex_opts_default(gf_simplex_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iter = 2000;
  o->oversample = 5;
  o->ftol = 1e-8;
  o->poll_every = 16;
  o->use_graph = 1;
}

gf_status gf_fit_simplex(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *data, const float *weight,
                         double *theta, const gf_simplex_opts *opts, gf_lm_result *res, double *trace, int trace_cap) {
  ProfBind pb_(c);
  if (!c || !b || !p || !data || !weight || !theta || !opts || !res || !opts->step)
    return fail(c, GF_EINVAL, "gf_fit_simplex: null argument (step is required)");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_fit_simplex: PSF prepared for another batch");
  gf_simplex_opts o = *opts;
  if (o.max_iter < 0 || o.oversample < 1 || o.oversample > GF_MAX_OVERSAMPLE || !(o.ftol >= 0.0) ||
      (trace && trace_cap < 1))
    return fail(c, GF_EINVAL, "gf_fit_simplex: invalid options");
  if (o.poll_every < 1) o.poll_every = 1;
  const int S = o.oversample;
  constexpr int kV = kMaxP + 1;
  double *X = nullptr, *F = nullptr, *XR = nullptr, *theta_t = nullptr;
  float *mpad = nullptr, *mconv = nullptr;
  float2 *S1 = nullptr, *S2 = nullptr, *cpart = nullptr;
  int *mask = nullptr, *cnt = nullptr;
  void *state = nullptr;
  auto layout = [&](Arena &ar) {
    X = ar.take<double>((int64_t)b->n * kV * kMaxP);
    F = ar.take<double>((int64_t)b->n * kV);
    XR = ar.take<double>((int64_t)b->n * kMaxP);
    theta_t = ar.take<double>(b->n_par);
    mpad = ar.take<float>(b->n_pad);
    mconv = ar.take<float>(b->n_pix);
    S1 = ar.take<float2>(p->n_s1);
    S2 = ar.take<float2>(p->n_s2);
    cpart = ar.take<float2>(chi2_slots(b, p));
    mask = ar.take<int>(b->n);
    cnt = ar.take<int>(16);
    state = ar.take<char>((int64_t)b->n * (int64_t)nm_state_bytes());
  };
  Arena a;
  layout(a);
  gf_status st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  layout(a);
  hipStream_t cs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  GF_TRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  GF_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(cs);   // graph launches may still be in flight
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    (void)hipEventDestroy(ev);
  };
  auto run = [&]() -> gf_status {
    GF_TRY(c, hipEventRecord(ev, c->stream));
    GF_TRY(c, hipStreamWaitEvent(cs, ev, 0));
    GF_TRY(c, launch_nm_init(cs, b, theta, o.step, &o, X, theta_t, state, mask, cnt));
    auto iteration = [&]() -> gf_status {
      GF_TRY(c, launch_nm_zero(cs, cnt));
      GF_TRY(c, launch_eval_d(cs, b, theta_t, S, c->d_bn, mpad, mask, nullptr));
      GF_TRY(c, conv_chi2(cs, b, p, mpad, S1, S2, mconv, theta_t, true, data, weight, cpart, mask, nullptr, &c->fork));
      GF_TRY(c, launch_nm_step(cs, b, p->d_c2_first, cpart, &o, state, X, F, XR, theta_t, mask, trace, trace_cap,
                               cnt));
      return GF_OK;
    };
    if (o.use_graph) {
      GF_TRY(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      gf_status s2 = iteration();
      hipError_t ce = hipStreamEndCapture(cs, &graph);
      if (s2 != GF_OK) return s2;
      GF_TRY(c, ce);
      GF_TRY(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    // every iteration costs at most P + 2 evaluations (reflection, expansion
    // or contraction, P shrink points), plus P + 1 for the initial simplex
    const int64_t max_evals = ((int64_t)o.max_iter + 1) * (b->max_P + 2) + b->max_P + 1;
    for (int64_t it = 0; it < max_evals; ++it) {
      if (exec) {
        GF_TRY(c, hipGraphLaunch(exec, cs));
      } else {
        gf_status s2 = iteration();
        if (s2 != GF_OK) return s2;
      }
      if ((it + 1) % o.poll_every == 0 || it + 1 == max_evals) {
        GF_TRY(c, hipMemcpyAsync(c->h_pinned, cnt, sizeof(int), hipMemcpyDeviceToHost, cs));
        GF_TRY(c, hipStreamSynchronize(cs));
        if (*(volatile int *)c->h_pinned == 0) break;
      }
    }
    GF_TRY(c, launch_nm_result(cs, b, state, F, X, theta, res));
    GF_TRY(c, hipEventRecord(ev, cs));
    GF_TRY(c, hipStreamWaitEvent(c->stream, ev, 0));
    return GF_OK;
  };
  st = run();
  cleanup();
  return st;
}

// ---------------------------------------------------------------- MCMC
void gf_mcmc_opts_default(gf_mcmc_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_steps = 1000;
  o->oversample = 5;
  o->thin = 1;
  o->use_graph = 1;
}

gf_status gf_mcmc_run(gf_ctx *c, const gf_batch *b, const gf_psf *p, const float *data, const float *weight,
                      double *theta, double *chi2, const gf_mcmc_opts *opts, float *samples, int32_t *accepted) {
  ProfBind pb_(c);
  if (!c || !b || !p || !data || !weight || !theta || !chi2 || !opts)
    return fail(c, GF_EINVAL, "gf_mcmc_run: null argument");
  if (p->batch != b) return fail(c, GF_EINVAL, "gf_mcmc_run: PSF prepared for another batch");
  const gf_mcmc_opts o = *opts;
  if (o.n_steps < 0 || o.thin < 1 || o.oversample < 1 || o.oversample > GF_MAX_OVERSAMPLE || o.step0 < 0)
    return fail(c, GF_EINVAL, "gf_mcmc_run: invalid options");
  const int S = o.oversample;
  Arena a;
  double *theta_t = nullptr, *chi2_d = nullptr;
  float *mpad = nullptr, *mconv = nullptr;
  float2 *S1 = nullptr, *S2 = nullptr, *cpart = nullptr, *pairs = nullptr;
  int *mask = nullptr;
  int64_t *tstep = nullptr;
  auto layout = [&](Arena &ar) {
    theta_t = ar.take<double>(b->n_par);
    mpad = ar.take<float>(b->n_pad);
    mconv = ar.take<float>(b->n_pix);
    S1 = ar.take<float2>(p->n_s1);
    S2 = ar.take<float2>(p->n_s2);
    cpart = ar.take<float2>(chi2_slots(b, p));
    pairs = ar.take<float2>(b->n);
    mask = ar.take<int>(b->n);
    tstep = ar.take<int64_t>(1);
    chi2_d = chi2;
  };
  layout(a);
  gf_status st = ensure_ws(c, a.off);
  if (st != GF_OK) return st;
  st = ensure_counters(c, b->n);
  if (st != GF_OK) return st;
  a = Arena{(char *)c->ws, 0};
  layout(a);
  hipStream_t cs = c->stream;
  // chi^2 of the start point
  GF_TRY(c, launch_eval_d(cs, b, theta, S, c->d_bn, mpad, nullptr, nullptr));
  GF_TRY(c, conv_chi2(cs, b, p, mpad, S1, S2, mconv, theta, true, data, weight, cpart, nullptr, nullptr, &c->fork));
  GF_TRY(c, launch_pair_final(cs, b->n, p->d_c2_first, cpart, pairs, nullptr));
  GF_TRY(c, launch_mcmc_init(cs, b->n, pairs, chi2_d, tstep));
  auto step = [&](hipStream_t sx) -> gf_status {
    GF_TRY(c, launch_mcmc_propose(sx, b, theta, o.scale, o.lo, o.hi, o.key0, o.key1, o.stream, o.step0, tstep,
                                  theta_t, mask));
    GF_TRY(c, launch_eval_d(sx, b, theta_t, S, c->d_bn, mpad, mask, nullptr));
    GF_TRY(c, conv_chi2(sx, b, p, mpad, S1, S2, mconv, theta_t, true, data, weight, cpart, mask, nullptr, &c->fork));
    GF_TRY(c, launch_mcmc_accept(sx, b, p->d_c2_first, cpart, mask, o.key0, o.key1, o.stream, o.step0, tstep, theta, theta_t, chi2_d,
                                 accepted, samples, o.thin));
    return GF_OK;
  };
  if (o.use_graph && o.n_steps > 1) {
    hipStream_t gs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GF_TRY(c, hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    gf_status r = GF_OK;
    auto body = [&]() -> gf_status {
      GF_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      GF_TRY(c, hipEventRecord(ev, cs));
      GF_TRY(c, hipStreamWaitEvent(gs, ev, 0));
      GF_TRY(c, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      gf_status s2 = step(gs);
      hipError_t ce = hipStreamEndCapture(gs, &graph);
      if (s2 != GF_OK) return s2;
      GF_TRY(c, ce);
      GF_TRY(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      for (int t = 0; t < o.n_steps; ++t) GF_TRY(c, hipGraphLaunch(exec, gs));
      GF_TRY(c, hipEventRecord(ev, gs));
      GF_TRY(c, hipStreamWaitEvent(cs, ev, 0));
      return GF_OK;
    };
    r = body();
    (void)hipStreamSynchronize(gs);   // graph launches may still be in flight
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(gs);
    if (ev) (void)hipEventDestroy(ev);
    return r;
  }
  for (int t = 0; t < o.n_steps; ++t) {
    gf_status r = step(cs);
    if (r != GF_OK) return r;
  }
  return GF_OK;
}

// ---------------------------------------------------------------- profiling
gf_status gf_profile_start(gf_ctx *c) {
  if (!c) return GF_EINVAL;
  GF_TRY(c, hipStreamSynchronize(c->stream));
  c->prof.recs.clear();
  c->prof.used = 0;
  c->prof.on = true;
  return GF_OK;
}

gf_status gf_profile_stop(gf_ctx *c) {
  if (!c) return GF_EINVAL;
  c->prof.on = false;
  return GF_OK;
}

int gf_profile_kernels(gf_ctx *c) {
  if (!c) return -1;
  for (const auto &r : c->prof.recs)
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
  std::vector<std::string> names;
  for (const auto &r : c->prof.recs)
    if (std::find(names.begin(), names.end(), r.name) == names.end()) names.push_back(r.name);
  return (int)names.size();
}

gf_status gf_profile_get(gf_ctx *c, int i, char *name, int name_cap, int64_t *launches, double *total_ms) {
  if (!c || i < 0) return GF_EINVAL;
  for (const auto &r : c->prof.recs) GF_TRY(c, hipEventSynchronize(r.b));
  std::vector<std::string> names;
  for (const auto &r : c->prof.recs)
    if (std::find(names.begin(), names.end(), r.name) == names.end()) names.push_back(r.name);
  if (i >= (int)names.size()) return fail(c, GF_EINVAL, "gf_profile_get: index out of range");
  int64_t n = 0;
  double tot = 0.0;
  for (const auto &r : c->prof.recs) {
    if (names[i] != r.name) continue;
    float ms = 0.0f;
    GF_TRY(c, hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++n;
  }
  if (name && name_cap > 0) {
    std::strncpy(name, names[i].c_str(), (size_t)name_cap - 1);
    name[name_cap - 1] = 0;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  return GF_OK;
}

}  // extern "C"

namespace gf {
// A batch of flat stamps (H*W values, P parameters each) for the cube path.
gf_status batch_create_flat(gf_ctx *c, int n, const int32_t *H, const int32_t *W, int P, gf_batch **out) {
  std::vector<int32_t> ones(n, 1);
  return create_batch(c, n, H, W, ones.data(), ones.data(), 0, nullptr, out, P);
}
}  // namespace gf

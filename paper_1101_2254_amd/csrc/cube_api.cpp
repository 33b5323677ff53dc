// cube_api.cpp -- host side of the data-cube family: cube batches, the model,
// chi^2, Jacobian and Levenberg-Marquardt entry points.  A cube batch keeps
// two image batches over the same cubes: `conv`, one H x W stamp per cube
// whose Nc (or 11 Nc) channels the spatial PSF convolution takes, and
// `flat`, one stamp of Nc H W voxels per cube with 12 parameters, on which
// chi^2, the normal equations and the LM state kernels of the image path
// run.  The convolution's channel layout (stamp offset times channels, then
// channel planes) makes its output the flat stamps' voxel layout, and the
// Jacobian's 11 channels per cube the channel layout of the normal
// equations.
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gf_internal.h"

namespace gf {
gf_status batch_create_flat(gf_ctx *c, int n, const int32_t *H, const int32_t *W, int P, gf_batch **out);
hipError_t launch_cube_eval(hipStream_t, const CubeDesc *, const Work *, int, const double *, const float4 *, int, int,
                            int, int, const int *, float *);
hipError_t launch_cube_jac(hipStream_t, const CubeDesc *, const Work *, int, const double *, const float4 *, int, int,
                           int, int, const int *, float *);
hipError_t launch_cube_lsf(hipStream_t, const CubeDesc *, const Work *, int, const float *, int, int, int, const int *,
                           const float *, float *);
hipError_t launch_cube_cont(hipStream_t, const gf_batch *, const double *, float *);
hipError_t launch_cube_jac_assemble(hipStream_t, const gf_batch *, const float *, float *);
hipError_t launch_cube_clip(hipStream_t, int64_t, const double *, const double *, const double *, double *);
hipError_t launch_fft_conv(hipStream_t, const gf_batch *, const gf_psf *, const float *, int, float2 *, float2 *,
                           float *, const int *, const WorkView *, const Chi2Epi *ep, const FftFork *fork);
hipError_t launch_direct(hipStream_t, const gf_batch *, const gf_psf *, const float *, int, float *, bool,
                         const int *, const WorkView *);
hipError_t launch_chi2(hipStream_t, const gf_batch *, const float *, const void *, bool, const float *,
                       const float *, float *, float2 *, unsigned int *, float2 *, const int *);
hipError_t launch_normal_eq(hipStream_t, const gf_batch *, const float *, const double *, const float *,
                            const float *, float *, int, int, const int *, const WorkView *, float2 *, int px,
                            const float *mie);
hipError_t launch_lm_init(hipStream_t, const gf_batch *, double, const int32_t *, const float2 *, LMState *, int *, int *,
                          int *, int model_ie);
hipError_t launch_lm_solve(hipStream_t, const gf_batch *, const float *, const gf_lm_opts *, LMState *, double *,
                           const double *, double *, int *, int *, int *, CompC *, CompC *, const float4 *,
                           const WorkView *, int px);
hipError_t launch_lm_update(hipStream_t, const gf_batch *, const gf_lm_opts *, const int32_t *, const float2 *,
                            LMState *, double *, const double *, int *, int *, int *, CompC *, CompC *,
                            const WorkView *, int model_ie);
hipError_t launch_lm_result(hipStream_t, int, const LMState *, gf_lm_result *);
}  // namespace gf

using namespace gf;

struct gf_cube_batch {
  gf_ctx *ctx = nullptr;
  int n = 0, Nc = 0, Kl = 0;
  std::vector<CubeDesc> h_desc;
  CubeDesc *d_desc = nullptr;
  std::vector<Work> h_sp;          // (cube, 256 padded spaxels)
  Work *d_sp = nullptr;
  int64_t n_pad = 0, n_pix = 0;    // spatial padded and plain spaxels of the batch
  std::vector<int64_t> vox_off, psf_off, lsf_off, par_off;
  gf_batch *conv = nullptr, *flat = nullptr;
  gf_psf *psf = nullptr;
  float *d_lsf = nullptr;
  float *d_psf = nullptr;          // the batch's copy of the PSF taps (the direct path reads them per call)
  void *ws = nullptr;
  size_t ws_bytes = 0;
};

namespace {

constexpr int kJ = 11;   // derivative channels of a cube (every parameter but the continuum)

gf_status cfail(gf_ctx *c, gf_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

#define CUBE_TRY(ctx, expr)                                                                                  \
  do {                                                                                                       \
    hipError_t e_ = (expr);                                                                                  \
    if (e_ != hipSuccess) return cfail(ctx, GF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Bump layout over the batch's workspace (sized on a first pass with base 0).
struct Lay {
  char *base = nullptr;
  size_t off = 0;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (size_t)std::max<int64_t>(n, 0);
    return p;
  }
};

struct CubeBufs {
  float *pad = nullptr;     // padded cubes: nk * Mc planes per cube
  float *lsf = nullptr;     // after the LSF: nk * Nc planes of the padded spatial grid
  float *conv = nullptr;    // after the PSF: nk * Nc H W per cube (flat layout)
  float2 *S1 = nullptr, *S2 = nullptr;
  float2 *part = nullptr;   // chi^2 partials (flat pixel-chunk slots)
  float2 *c2 = nullptr;     // per-cube (hi, lo)
  float *npart = nullptr;   // Gram partials
  double *Ag = nullptr, *theta_t = nullptr;
  LMState *st = nullptr;
  int *mjac = nullptr, *mtrial = nullptr, *cnt = nullptr;
  float *model = nullptr;   // LM: the convolved model of the last trial (flat layout), whose Ie column it gives
};

void layout(const gf_cube_batch *cb, int nk, bool lm, Lay &a, CubeBufs &B) {
  const int Mc = cb->Nc + cb->Kl - 1;
  B.pad = a.take<float>(cb->n_pad * Mc * nk);
  B.lsf = a.take<float>(cb->n_pad * cb->Nc * nk);
  B.conv = a.take<float>(cb->n_pix * cb->Nc * nk);
  B.S1 = a.take<float2>(cb->psf->n_s1 * cb->Nc * nk);
  B.S2 = a.take<float2>(cb->psf->n_s2 * cb->Nc * nk);
  B.part = a.take<float2>((int64_t)cb->flat->h_pix.size());
  B.c2 = a.take<float2>(cb->n);
  if (!lm) return;
  B.npart = a.take<float>((int64_t)cb->flat->h_neq.size() * 256);
  B.Ag = a.take<double>((int64_t)cb->n * (kMaxP * kMaxP + kMaxP));
  B.theta_t = a.take<double>((int64_t)cb->n * GF_CUBE_NPAR);
  B.st = a.take<LMState>(cb->n);
  B.mjac = a.take<int>(cb->n);
  B.mtrial = a.take<int>(cb->n);
  B.cnt = a.take<int>(1);
  B.model = a.take<float>(cb->n_pix * cb->Nc);
}

gf_status buffers(gf_ctx *c, gf_cube_batch *cb, int nk, bool lm, CubeBufs &B) {
  Lay a;
  layout(cb, nk, lm, a, B);
  if (a.off > cb->ws_bytes) {
    if (cb->ws) {
      CUBE_TRY(c, hipStreamSynchronize(c->stream));
      (void)hipFree(cb->ws);
      cb->ws = nullptr;
      cb->ws_bytes = 0;
    }
    CUBE_TRY(c, hipMalloc(&cb->ws, a.off));
    cb->ws_bytes = a.off;
  }
  a = Lay{(char *)cb->ws, 0};
  layout(cb, nk, lm, a, B);
  return GF_OK;
}

gf_status check(gf_ctx *c, const gf_cube_batch *cb, int S, int Sv, const char *what) {
  if (!c || !cb) return cfail(c, GF_EINVAL, std::string(what) + ": null argument");
  if (cb->ctx != c) return cfail(c, GF_EINVAL, std::string(what) + ": cube batch of another context");
  if (!cb->psf) return cfail(c, GF_EINVAL, std::string(what) + ": gf_cube_set_kernels has not been called");
  if (S < 1 || S > GF_MAX_OVERSAMPLE || Sv < 1 || Sv > GF_MAX_OVERSAMPLE)
    return cfail(c, GF_EINVAL, std::string(what) + ": oversample out of range");
  return GF_OK;
}

// Steps 1-2 of every cube in mask (nk = 1: the model without continuum into
// out) or of their 11 derivative channels (nk = 11; with kMaskModelIe in a
// cube's mask all but the Ie block).
gf_status steps12(gf_ctx *c, gf_cube_batch *cb, hipStream_t st, const double *theta, int S, int Sv, int nk,
                  const int *mask, const CubeBufs &B, float *out) {
  const int nw = (int)cb->h_sp.size();
  if (nk == 1)
    CUBE_TRY(c, launch_cube_eval(st, cb->d_desc, cb->d_sp, nw, theta, c->d_bn, cb->Nc, cb->Kl, S, Sv, mask, B.pad));
  else
    CUBE_TRY(c, launch_cube_jac(st, cb->d_desc, cb->d_sp, nw, theta, c->d_bn, cb->Nc, cb->Kl, S, Sv, mask, B.pad));
  CUBE_TRY(c, launch_cube_lsf(st, cb->d_desc, cb->d_sp, nw, cb->d_lsf, cb->Nc, cb->Kl, nk, mask, B.pad, B.lsf));
  const int nch = nk * cb->Nc;
  CUBE_TRY(c, launch_fft_conv(st, cb->conv, cb->psf, B.lsf, nch, B.S1, B.S2, out, mask, nullptr, nullptr, &c->fork));
  CUBE_TRY(c, launch_direct(st, cb->conv, cb->psf, B.lsf, nch, out, false, mask, nullptr));
  return GF_OK;
}

}  // namespace

extern "C" {

gf_status gf_cube_batch_create(gf_ctx *c, int n, const int32_t *H, const int32_t *W, const int32_t *K, int n_chan,
                               int K_lsf, gf_cube_batch **out) {
  if (!c || !out || !H || !W || !K) return cfail(c, GF_EINVAL, "gf_cube_batch_create: null argument");
  *out = nullptr;
  if (n < 1) return cfail(c, GF_EINVAL, "gf_cube_batch_create: n < 1");
  if (n_chan < 1 || n_chan > GF_CUBE_MAX_CHAN || K_lsf < 1 || K_lsf > GF_LINE_MAX_K || (K_lsf % 2) == 0)
    return cfail(c, GF_ESHAPE, "gf_cube_batch_create: need 1 <= n_chan <= GF_CUBE_MAX_CHAN and odd K_lsf in 1..GF_LINE_MAX_K");
  gf_cube_batch *cb = new (std::nothrow) gf_cube_batch();
  if (!cb) return cfail(c, GF_ENOMEM, "gf_cube_batch_create: host allocation");
  cb->ctx = c;
  cb->n = n;
  cb->Nc = n_chan;
  cb->Kl = K_lsf;
  cb->h_desc.resize(n);
  std::vector<int32_t> nc(n, 1), fh(n), fw(n);
  int64_t psf = 0;
  for (int s = 0; s < n; ++s) {
    if (H[s] < 1 || W[s] < 1 || K[s] < 1 || (K[s] % 2) == 0 || K[s] > GF_MAX_K || H[s] + K[s] - 1 > GF_MAX_FFT ||
        W[s] + K[s] - 1 > GF_MAX_FFT || (int64_t)n_chan * H[s] * W[s] > (1LL << 30)) {
      delete cb;
      return cfail(c, GF_ESHAPE, "gf_cube_batch_create: unsupported shape for cube " + std::to_string(s));
    }
    CubeDesc &d = cb->h_desc[s];
    d.H = H[s];
    d.W = W[s];
    d.K = K[s];
    d.Mh = H[s] + K[s] - 1;
    d.Mw = W[s] + K[s] - 1;
    d.pad0 = 0;
    d.pad = cb->n_pad;
    d.pix = cb->n_pix;
    d.par = (int64_t)s * GF_CUBE_NPAR;
    d.lsf = (int64_t)s * K_lsf;
    cb->vox_off.push_back(cb->n_pix * n_chan);
    cb->psf_off.push_back(psf);
    cb->lsf_off.push_back(d.lsf);
    cb->par_off.push_back(d.par);
    const int nu = (d.Mh * d.Mw + kThreads - 1) / kThreads;
    for (int u = 0; u < nu; ++u) cb->h_sp.push_back({s, u});
    cb->n_pad += (int64_t)d.Mh * d.Mw;
    cb->n_pix += (int64_t)d.H * d.W;
    psf += (int64_t)K[s] * K[s];
    // the flat stamp: Nc rows of H W voxels
    fh[s] = n_chan;
    fw[s] = H[s] * W[s];
  }
  cb->vox_off.push_back(cb->n_pix * n_chan);
  cb->psf_off.push_back(psf);
  cb->lsf_off.push_back((int64_t)n * K_lsf);
  cb->par_off.push_back((int64_t)n * GF_CUBE_NPAR);
  gf_status st = gf_batch_create(c, n, H, W, K, nc.data(), 0, &cb->conv);
  if (st == GF_OK) st = batch_create_flat(c, n, fh.data(), fw.data(), GF_CUBE_NPAR, &cb->flat);
  if (st != GF_OK) {
    gf_cube_batch_destroy(cb);
    return st;
  }
  hipError_t e = hipMalloc((void **)&cb->d_desc, sizeof(CubeDesc) * (size_t)n);
  if (e == hipSuccess)
    e = hipMemcpy(cb->d_desc, cb->h_desc.data(), sizeof(CubeDesc) * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void **)&cb->d_sp, sizeof(Work) * cb->h_sp.size());
  if (e == hipSuccess)
    e = hipMemcpy(cb->d_sp, cb->h_sp.data(), sizeof(Work) * cb->h_sp.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void **)&cb->d_lsf, sizeof(float) * (size_t)n * K_lsf);
  if (e == hipSuccess) e = hipMalloc((void **)&cb->d_psf, sizeof(float) * (size_t)psf);
  if (e != hipSuccess) {
    gf_cube_batch_destroy(cb);
    return cfail(c, GF_EDEVICE, std::string("gf_cube_batch_create: ") + hipGetErrorString(e));
  }
  *out = cb;
  return GF_OK;
}

void gf_cube_batch_destroy(gf_cube_batch *cb) {
  if (!cb) return;
  if (cb->psf) gf_psf_destroy(cb->psf);
  if (cb->conv) gf_batch_destroy(cb->conv);
  if (cb->flat) gf_batch_destroy(cb->flat);
  if (cb->d_desc) (void)hipFree(cb->d_desc);
  if (cb->d_sp) (void)hipFree(cb->d_sp);
  if (cb->d_lsf) (void)hipFree(cb->d_lsf);
  if (cb->d_psf) (void)hipFree(cb->d_psf);
  if (cb->ws) (void)hipFree(cb->ws);
  delete cb;
}

gf_status gf_cube_batch_offsets(const gf_cube_batch *cb, int64_t *vox_off, int64_t *psf_off, int64_t *lsf_off,
                                int64_t *par_off) {
  if (!cb) return GF_EINVAL;
  for (int s = 0; s <= cb->n; ++s) {
    if (vox_off) vox_off[s] = cb->vox_off[s];
    if (psf_off) psf_off[s] = cb->psf_off[s];
    if (lsf_off) lsf_off[s] = cb->lsf_off[s];
    if (par_off) par_off[s] = cb->par_off[s];
  }
  return GF_OK;
}

gf_status gf_cube_set_kernels(gf_ctx *c, gf_cube_batch *cb, const float *psf, const float *lsf, int conv_mode) {
  if (!c || !cb || !psf || !lsf) return cfail(c, GF_EINVAL, "gf_cube_set_kernels: null argument");
  if (cb->ctx != c) return cfail(c, GF_EINVAL, "gf_cube_set_kernels: cube batch of another context");
  if (cb->psf) {
    CUBE_TRY(c, hipStreamSynchronize(c->stream));
    gf_psf_destroy(cb->psf);
    cb->psf = nullptr;
  }
  CUBE_TRY(c, hipMemcpyAsync(cb->d_psf, psf, sizeof(float) * (size_t)cb->psf_off[cb->n], hipMemcpyDeviceToDevice,
                             c->stream));
  CUBE_TRY(c, hipMemcpyAsync(cb->d_lsf, lsf, sizeof(float) * (size_t)cb->n * cb->Kl, hipMemcpyDeviceToDevice,
                             c->stream));
  return gf_psf_prepare(c, cb->conv, cb->d_psf, conv_mode, &cb->psf);
}

gf_status gf_cube_model(gf_ctx *c, gf_cube_batch *cb, const double *theta, int S, int Sv, float *out) {
  ProfBind pb_(c);
  gf_status st = check(c, cb, S, Sv, "gf_cube_model");
  if (st != GF_OK) return st;
  if (!theta || !out) return cfail(c, GF_EINVAL, "gf_cube_model: null argument");
  CubeBufs B;
  st = buffers(c, cb, 1, false, B);
  if (st != GF_OK) return st;
  B.conv = out;
  st = steps12(c, cb, c->stream, theta, S, Sv, 1, nullptr, B, B.conv);
  if (st != GF_OK) return st;
  CUBE_TRY(c, launch_cube_cont(c->stream, cb->flat, theta, out));
  return GF_OK;
}

gf_status gf_cube_chi2(gf_ctx *c, gf_cube_batch *cb, const double *theta, int S, int Sv, const float *data,
                       const float *weight, float *chi2) {
  ProfBind pb_(c);
  gf_status st = check(c, cb, S, Sv, "gf_cube_chi2");
  if (st != GF_OK) return st;
  if (!theta || !data || !weight || !chi2) return cfail(c, GF_EINVAL, "gf_cube_chi2: null argument");
  CubeBufs B;
  st = buffers(c, cb, 1, false, B);
  if (st != GF_OK) return st;
  st = steps12(c, cb, c->stream, theta, S, Sv, 1, nullptr, B, B.conv);
  if (st != GF_OK) return st;
  CUBE_TRY(c, launch_chi2(c->stream, cb->flat, B.conv, theta, true, data, weight, nullptr, B.part, nullptr,
                          (float2 *)chi2, nullptr));
  return GF_OK;
}

gf_status gf_cube_jacobian(gf_ctx *c, gf_cube_batch *cb, const double *theta, int S, int Sv, float *out) {
  ProfBind pb_(c);
  gf_status st = check(c, cb, S, Sv, "gf_cube_jacobian");
  if (st != GF_OK) return st;
  if (!theta || !out) return cfail(c, GF_EINVAL, "gf_cube_jacobian: null argument");
  CubeBufs B;
  st = buffers(c, cb, kJ, false, B);
  if (st != GF_OK) return st;
  st = steps12(c, cb, c->stream, theta, S, Sv, kJ, nullptr, B, B.conv);
  if (st != GF_OK) return st;
  CUBE_TRY(c, launch_cube_jac_assemble(c->stream, cb->flat, B.conv, out));
  return GF_OK;
}

gf_status gf_cube_fit_lm(gf_ctx *c, gf_cube_batch *cb, const float *data, const float *weight, double *theta,
                         const gf_lm_opts *opts, int Sv, gf_lm_result *res) {
  ProfBind pb_(c);
  gf_lm_opts o;
  if (opts) o = *opts; else gf_lm_opts_default(&o);
  if (opts && opts->struct_size != (int32_t)sizeof(gf_lm_opts))
    return cfail(c, GF_EINVAL, "gf_cube_fit_lm: opts->struct_size differs from sizeof(gf_lm_opts) (initialise with gf_lm_opts_default)");
  gf_status st = check(c, cb, o.oversample, Sv, "gf_cube_fit_lm");
  if (st != GF_OK) return st;
  if (!data || !weight || !theta || !res) return cfail(c, GF_EINVAL, "gf_cube_fit_lm: null argument");
  if (o.max_iter < 0 || !(o.lambda_up > 1.0) || !(o.lambda_down > 1.0) || !(o.lambda0 > 0.0))
    return cfail(c, GF_EINVAL, "gf_cube_fit_lm: invalid options");
  if (o.poll_every < 1) o.poll_every = 1;
  CubeBufs B;
  st = buffers(c, cb, kJ, true, B);
  if (st != GF_OK) return st;
  const int S = o.oversample;
  hipStream_t cs = c->stream;
  gf_batch *fb = cb->flat;
  const int64_t np = (int64_t)cb->n * GF_CUBE_NPAR;
  // start: clip, evaluate, chi^2
  CUBE_TRY(c, launch_cube_clip(cs, np, o.start ? o.start : theta, o.lo, o.hi, theta));
  st = steps12(c, cb, cs, theta, S, Sv, 1, nullptr, B, B.model);
  if (st != GF_OK) return st;
  CUBE_TRY(c, launch_chi2(cs, fb, B.model, theta, true, data, weight, nullptr, B.part, nullptr, B.c2, nullptr));
  // the Jacobian masks flag every cube: its Ie column comes from the kept model
  CUBE_TRY(c, launch_lm_init(cs, fb, o.lambda0, fb->d_pix_first, B.part, B.st, B.mjac, B.mtrial, B.cnt, cb->Nc));
  for (int it = 0; it < o.max_iter; ++it) {
    // Jacobian of the cubes that need one, their normal equations
    st = steps12(c, cb, cs, theta, S, Sv, kJ, B.mjac, B, B.conv);
    if (st != GF_OK) return st;
    CUBE_TRY(c, launch_normal_eq(cs, fb, B.conv, theta, data, weight, B.npart, 256, kJ, B.mjac, nullptr, nullptr,
                                 kCubePX, B.model));
    CUBE_TRY(c, launch_lm_solve(cs, fb, B.npart, &o, B.st, B.Ag, theta, B.theta_t, B.mjac, B.mtrial, B.cnt, nullptr,
                                nullptr, c->d_bn, nullptr, kCubePX));
    // trial point: model, chi^2, accept or reject
    st = steps12(c, cb, cs, B.theta_t, S, Sv, 1, B.mtrial, B, B.model);
    if (st != GF_OK) return st;
    CUBE_TRY(c, launch_chi2(cs, fb, B.model, B.theta_t, true, data, weight, nullptr, B.part, nullptr, B.c2,
                            B.mtrial));
    CUBE_TRY(c, launch_lm_update(cs, fb, &o, fb->d_pix_first, B.part, B.st, theta, B.theta_t, B.mjac, B.mtrial,
                                 B.cnt, nullptr, nullptr, nullptr, cb->Nc));
    if ((it + 1) % o.poll_every == 0 || it + 1 == o.max_iter) {
      CUBE_TRY(c, hipMemcpyAsync(c->h_pinned, B.cnt, sizeof(int), hipMemcpyDeviceToHost, cs));
      CUBE_TRY(c, hipStreamSynchronize(cs));
      if (*c->h_pinned == 0) break;
    }
  }
  CUBE_TRY(c, launch_lm_result(cs, cb->n, B.st, res));
  return GF_OK;
}

}  // extern "C"

// gf_internal.h -- structures shared by the host side and the HIP kernels of
// libgf (the MI355X galaxy-fitting hot path).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gf.h"

namespace gf {

constexpr int kNPC = GF_NPC;
constexpr int kMaxComp = GF_MAX_COMP;
constexpr int kMaxP = kNPC * kMaxComp + 1;
constexpr int kThreads = 256;          // threads per workgroup for pixel kernels (4 wave64)
constexpr int kEvalTile = 256;         // padded pixels per eval workgroup (one per thread)
constexpr int kPixChunk = 4096;        // pixels per chi^2 workgroup (16 per thread)
constexpr int kNeqChunk = 1024;        // pixels per normal-equation unit (one partial Gram matrix)
// Stamps of at least this many pixels have each unit summed by an
// eight-wave Gram workgroup (128 pixels per wave), smaller stamps by a
// four-wave one (256 per wave).  The split is a property of the stamp, so a
// stamp's partials do not depend on the batch.
constexpr int kNeqBigPix = 1 << 17;
// Parameters of a data cube after the continuum (v0, vproj, rt, sigma_v).
constexpr int kCubePX = 4;
// Complex values in the FFT LDS buffer of a workgroup (T*L <= this).  The
// kernels built for plan radices up to 18 or up to 24 need fewer registers;
// with their smaller buffers five workgroups fit on a CU instead of four
// (for the radix-24 build up to L = 576).
constexpr int kFftCap = 3840;
constexpr int kFftCapSmall = 3456;
constexpr int kFftCapMid = 3408;
constexpr int fft_cap(int rmax) { return rmax <= 18 ? kFftCapSmall : rmax <= 24 ? kFftCapMid : kFftCap; }
constexpr int kLmLanes = 2;           // lanes of a large plain-form LM fit
constexpr int kFftMaxStages = 12;
constexpr int kFftNarrowT = 1;         // row pairs per workgroup in the narrow launch shape
constexpr int kFftNarrowC = 2;         // bins per workgroup in the narrow launch shape
constexpr int kDirectTH = 16;          // direct convolution output tile rows
constexpr int kDirectTW = 64;          // direct convolution output tile columns
constexpr int kDirectMaxK = 41;        // largest PSF side on the direct path

// b_n table: nodes n_i = kBnLo + i*h, i = -2 .. kBnNodes+1 (two guard nodes at
// each end for the difference stencils); the device copy holds
// (b_n, db_n/dn, d2b_n/dn2, 0) per node.
constexpr double kBnLo = 0.2;
constexpr double kBnHi = 10.0;
constexpr int kBnNodes = 4097;

// Per-stamp geometry and flat-array offsets.
struct StampDesc {
  int32_t H, W, K, ncomp;
  int32_t Mh, Mw, P, pad0;
  int64_t pix, pad, psf, par, img, jac;
};

// Per-stamp convolution path chosen by gf_psf_prepare.
struct PathDesc {
  int32_t fft;    // 0 = direct, 1 = multi-pass FFT, 2 = one-workgroup FFT (fused)
  int32_t L;      // FFT side (0 on the direct path)
  int32_t plan;   // index into the plan table (-1 on the direct path)
  int32_t tw;     // offset of the side's twiddles exp(-2 pi i k / L) in the twiddle table
  int64_t otf;    // offset of this stamp's OTF (complex elements), in the layout of its form
  int64_t otf_mp; // offset of its OTF bin-major [L/2+1][L] for the multi-pass kernels (= otf on that form)
};

// Mixed-radix Stockham plan for one FFT side L (radix-r stage s works on
// sub-transforms of size ns[s]; nb = L / r butterflies per transform).
struct FftPlan {
  int32_t L, nstages, tw_off, pad0;
  int32_t radix[kFftMaxStages];
  int32_t ns[kFftMaxStages];
  uint32_t ns_magic[kFftMaxStages];
  uint32_t nb_magic[kFftMaxStages];
};

// Unit of work of a launch: (stamp, unit within the stamp).
struct Work {
  int32_t stamp;
  int32_t unit;
};

// What an FFT convolution launch computes: the valid convolution of the
// padded model (CONV), the adjoint correlation of an image onto the padded
// grid (CORR), the OTF of the PSF taps (OTF), or CONV ending in the chi^2
// epilogue instead of writing the model (CHI2).
enum { MODE_CONV = 0, MODE_CORR = 1, MODE_OTF = 2, MODE_CHI2 = 3 };

// FFT sides that the one-workgroup 2-D convolution covers: every even
// 2^a 3^b 5^c up to 192, whose half spectrum (L + 1 rows of L/2 + 1 bins,
// one padding slot per 32) fits one workgroup's LDS.
constexpr int kF2dSides[] = {8,  10, 12, 16, 18, 20,  24,  30,  32,  36,  40,  48,  50,  54,  60,
                             64, 72, 80, 90, 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192};
constexpr int kF2dN = (int)(sizeof(kF2dSides) / sizeof(kF2dSides[0]));
constexpr int kF2dMaxL = 192;
inline int f2d_class(int L) {
  for (int i = 0; i < kF2dN; ++i)
    if (kF2dSides[i] == L) return i;
  return -1;
}
// The side classes are launched in five buckets of similar LDS size (one
// launch per bucket covers every stamp of its sides): classes
// [kF2dBucketEnd[b-1], kF2dBucketEnd[b]), i.e. sides up to 64, 96, 128, 160
// and 192.
constexpr int kF2dBuckets = 5;
constexpr int kF2dBucketEnd[kF2dBuckets] = {16, 20, 24, 27, 30};
constexpr int f2d_bucket(int cls) {
  return cls < kF2dBucketEnd[0] ? 0 : cls < kF2dBucketEnd[1] ? 1 : cls < kF2dBucketEnd[2] ? 2
                                                           : cls < kF2dBucketEnd[3] ? 3 : 4;
}

// Work lists of one launch set: by default a batch's and a prepared PSF's
// full lists; gf_fit_lm substitutes lists that hold only the stamps still
// iterating, so finished stamps cost no workgroups.  Null pointers mean
// "the full list".
struct WorkView {
  const Work *eval = nullptr, *pix = nullptr, *neq = nullptr;
  int n_eval = 0, n_pix = 0, n_neq = 0, n_neq_big = 0;   // neq: the large stamps' units first
  const Work *rows = nullptr, *cols = nullptr, *irows = nullptr;
  int n_rows = 0, n_cols = 0, n_irows = 0;
  const Work *rows_n = nullptr, *cols_n = nullptr, *irows_n = nullptr;
  int n_rows_n = 0, n_cols_n = 0, n_irows_n = 0;
  const Work *direct = nullptr;
  int n_direct = 0;
  const Work *pix_direct = nullptr;
  int n_pix_direct = 0;
  const Work *stamps = nullptr;   // the stamps still iterating (unit 0), for the per-stamp LM kernels
  int n_stamps = 0;
  // one-workgroup FFT convolutions: entries of bucket b at
  // f2d[f2d_first[b] .. f2d_first[b + 1]) (unit = bucket)
  const Work *f2d = nullptr;
  int f2d_first[kF2dBuckets + 1] = {};
};

// Runs of consecutive entries of one stamp in a full work list, in list
// order (an LM fit restricts its lists to the stamps still iterating run by
// run).
struct ListRuns {
  std::vector<int32_t> stamp, beg, len;
};
// One contiguous piece of a restricted work list: len entries from src to
// dst + dst_off.
struct CopyRun {
  const Work *src;
  int64_t dst_off;
  int32_t len, pad0;
};

// One data cube: its spatial geometry and offsets (the spectral length Nc
// and LSF length Kl are those of the batch).
struct CubeDesc {
  int32_t H, W, K, Mh, Mw, pad0;
  int64_t pad;   // spatial padded offset: sum of Mh*Mw over the earlier cubes
  int64_t pix;   // spatial offset: sum of H*W
  int64_t par;   // parameter offset (GF_CUBE_NPAR per cube)
  int64_t lsf;   // LSF tap offset
};

// Per-component constants of the evaluation kernels (computed per workgroup).
struct CompC {
  int32_t ix, iy;    // integer part of the centre
  float fx, fy;      // centre minus integer part
  float ox[GF_MAX_OVERSAMPLE], oy[GF_MAX_OVERSAMPLE];  // sub-sample offset minus (fx, fy)
  float cs, sn;      // cos phi, sin phi
  float cq, sq;      // cos phi / q, sin phi / q
  float iq2;         // 1/q^2
  float a1, a0;      // t = exp2(a1 * log2(R^2) + a0)
  float b1;          // b_n * log2(e)
  float lie;         // log2(Ie)
  float ie, re, n, q, bn, dbn;
  float inv_n, inv_re, inv_q;
};

// chi^2 epilogue of the inverse-row FFT pass: the residuals of the convolved
// model against the observation are reduced where the model rows leave LDS,
// one compensated (hi, lo) partial per output row pair, and the model image
// itself is not written.
struct Chi2Epi {
  const float *data, *weight;
  const void *theta;        // sky of stamp s at theta[par + 7 ncomp]
  int32_t theta_f64;        // theta is double (else float)
  const int32_t *first;     // first partial slot of each stamp
  float2 *part;
  // when non-null: the convolved model of each one-component stamp (without
  // the sky) is also written, at model + its pixel offset
  float *model = nullptr;
};

// A Jacobian mask value with this bit set (one-component stamps of an LM fit
// in the plain form, and the cubes of a cube fit): the Ie channels are not
// evaluated or convolved, and the normal equations take that column from the
// convolved model of the same point, which the accepted trial's chi^2 pass
// left in the model buffer (the model is linear in Ie: dm/dIe = (m - sky) /
// Ie).  Bits 8 and up hold the channels per parameter (1 for an image, the
// spectral channels for a cube), so the Ie channels are those of parameter 2.
constexpr int kMaskModelIe = 2;
constexpr int kMaskCppShift = 8;
__device__ __host__ inline int mask_model_ie(int cpp) { return 1 | kMaskModelIe | (cpp << kMaskCppShift); }
__device__ __host__ inline bool skip_ie(const int *mask, int s, int ch) {
  if (!mask) return false;
  const int m = mask[s];
  const int cpp = m >> kMaskCppShift;
  return (m & kMaskModelIe) && ch >= 2 * cpp && ch < 3 * cpp;
}

// One spectrum of a line batch.
struct LineDesc {
  int32_t N, K, nl, pad0;
  int64_t data, lsf, par;   // offsets into the flat data / LSF / parameter arrays
};

// Options of the line fits, as passed to the device.
struct LineLMParams {
  int32_t max_iter, S;
  double lambda0, lambda_up, lambda_down, lambda_max, ftol, xtol;
  const double *lo, *hi;
  const uint8_t *free_mask;
};

// LM per-stamp state (device).
struct LMState {
  double lambda;
  double chi2;        // chi^2 at theta
  double chi2_trial;
  int32_t iters, nfev, njev, status, reason;
  int32_t active;     // still iterating
  int32_t need_jac;   // Jacobian at theta not yet formed
  int32_t trial;      // a trial point was produced this iteration
};

// BF16 values are stored as raw 16-bit words.
typedef uint16_t bf16_t;

// Epilogue of the BF16 GEMM: v = acc (+ bias[n]) (ReLU) (zero where
// mask(m, n) <= 0), stored to FP32 and/or BF16 outputs.
struct Epi {
  const float *bias;      // [N] or null
  int relu;
  const bf16_t *mask;     // null: no mask
  int ldm;
  float *outf;            // FP32 output or null
  int ldf;
  bf16_t *outb;           // BF16 output or null
  int ldb;
};

// Fast division by a runtime constant d (x, d < 2^16): m = ceil(2^32/d), m = 0 for d = 1.
inline uint32_t magic_for(uint32_t d) {
  return d <= 1 ? 0u : (uint32_t)(((1ull << 32) + d - 1) / d);
}

// ---------------------------------------------------------------- profiling
// Optional per-launch timing with HIP events recorded on the launching
// stream around each kernel (never inside a graph capture).  Entry points
// bind their context's profiler to the calling thread; launchers open a
// ProfScope named after the kernel.
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};

struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

extern thread_local Profiler *t_prof;

struct ProfScope {
  Profiler *p = nullptr;
  hipStream_t s = nullptr;
  ProfRec r{};
  ProfScope(hipStream_t st, const char *name) : s(st) {
    if (!t_prof || !t_prof->on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    r.name = name;
    r.a = t_prof->get();
    r.b = t_prof->get();
    if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) return;
    p = t_prof;
  }
  ~ProfScope() {
    if (!p) return;
    if (hipEventRecord(r.b, s) == hipSuccess) p->recs.push_back(r);
  }
};

}  // namespace gf

namespace gf {
// What one captured LM iteration depends on besides the context: the batch
// and PSF (their launch grids and device lists, by unique id, so an object
// freed and replaced at the same address does not match), the caller's
// pointers, the workspace, and the options that reach the kernels.
struct LmGraphKey {
  uint64_t batch_uid = 0, psf_uid = 0;
  const void *data = nullptr, *weight = nullptr, *theta = nullptr, *ws = nullptr;
  const void *lo = nullptr, *hi = nullptr, *free_mask = nullptr;
  int32_t max_iter = 0, oversample = 0, spec = 0;
  double lambda_up = 0, lambda_down = 0, lambda_max = 0, ftol = 0, xtol = 0;
  bool operator==(const LmGraphKey &o) const {
    return batch_uid == o.batch_uid && psf_uid == o.psf_uid && data == o.data && weight == o.weight &&
           theta == o.theta && ws == o.ws && lo == o.lo && hi == o.hi && free_mask == o.free_mask &&
           max_iter == o.max_iter && oversample == o.oversample && spec == o.spec && lambda_up == o.lambda_up &&
           lambda_down == o.lambda_down && lambda_max == o.lambda_max && ftol == o.ftol && xtol == o.xtol;
  }
};
// Process-wide unique, nonzero id for batches and PSFs.
uint64_t next_uid();

// Side streams and their fork and join events: launch_fft_conv runs the
// one-workgroup FFT buckets on the side streams (bucket b on lane
// kForkLane[b]) while the multi-pass stamps run on the caller's stream (all
// of them touch disjoint stamps), and joins before it returns, so the tail
// of each launch overlaps the others.  Null streams run everything on the
// caller's stream.  With the caller's stream, four streams in all: the
// hardware queues a process gets by default.
constexpr int kForkLanes = 3;
constexpr int kForkLane[kF2dBuckets] = {2, 2, 1, 0, 0};
struct FftFork {
  hipStream_t side[kForkLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kForkLanes] = {};
};
}  // namespace gf


// ---------------------------------------------------------------- host objects
struct gf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  float4 *d_bn = nullptr;      // b_n table (kBnNodes entries)
  unsigned int *d_counters = nullptr;  // self-resetting completion counters
  int64_t n_counters = 0;
  void *ws = nullptr;          // grow-only workspace
  size_t ws_bytes = 0;
  int *h_pinned = nullptr;     // pinned host word for LM polling
  void *h_states = nullptr;    // pinned copy of the LM states at a restriction (grown on demand)
  size_t h_states_bytes = 0;
  gf::Profiler prof;
  // side streams (default priority) and fork/join events for launches that
  // run concurrently, e.g. the per-line-count kernels of a line fit
  hipStream_t side[GF_LINE_MAX_LINES] = {};
  hipEvent_t side_ev[GF_LINE_MAX_LINES + 1] = {};
  // the one-workgroup FFT launches of a convolution run on this stream
  // beside the multi-pass launches of the same convolution (created with
  // the context, so a captured LM iteration can fork onto it)
  gf::FftFork fork{};
  // LM fits: their stream and join event, and the last captured iteration
  // graph with what it was captured for (replayed while the key matches)
  hipStream_t lm_stream = nullptr;
  hipEvent_t lm_ev = nullptr;
  // the second lane of a large plain-form fit (its stream) and the lanes'
  // poll events
  hipStream_t lm_lane_stream[gf::kLmLanes - 1] = {};   // lanes 1.. of a large LM fit
  hipEvent_t lm_lane_ev[gf::kLmLanes] = {};
  gf::LmGraphKey lm_key;
  hipGraph_t lm_graph = nullptr;
  hipGraphExec_t lm_exec = nullptr;
  // tuning table: per one-workgroup side class, the FFT form that the
  // automatic path choice takes (-1 untuned, 1 multi-pass, 2 one-workgroup)
  int8_t tune_form[gf::kF2dN];
  // per bucket of one-workgroup sides: the fewest still-fitting stamps for
  // which gf_fit_lm keeps that form (below it, they move to the multi-pass
  // launches)
  int32_t f2d_min_active[gf::kF2dBuckets];
  int8_t tune_min_done[gf::kF2dBuckets] = {};   // f2d_min_active measured (or read) for the bucket
  std::string tune_path;      // file the table is read from and written to ("" = no measuring)
  // PSF sides up to this are convolved directly by GF_CONV_AUTO
  int32_t tune_direct_k = 7;
  int8_t tune_direct_done = 0;   // measured (or read) for this context
  gf_ctx() {
    for (int i = 0; i < gf::kF2dN; ++i) tune_form[i] = -1;
    // eight rounds of workgroups on 256 CUs for a seven-channel Jacobian,
    // at the workgroups per CU each bucket's kernel fits (on the uneven
    // batch, keeping the form down to two rounds ran 2 % slower than the
    // multi-pass form alone, eight or more rounds 0.5 % faster)
    const int wg_per_cu[gf::kF2dBuckets] = {6, 3, 1, 1, 1};
    for (int b = 0; b < gf::kF2dBuckets; ++b) f2d_min_active[b] = 8 * 256 * wg_per_cu[b] / 7;
  }
};

namespace gf {
// Tuning table I/O and measurement (tune.cpp).
gf_status tune_load(gf_ctx *c);
gf_status tune_save(gf_ctx *c);
gf_status tune_side(gf_ctx *c, int L);
gf_status tune_direct(gf_ctx *c);
// Binds a context's profiler to the calling thread for one entry point.
struct ProfBind {
  Profiler *prev;
  explicit ProfBind(gf_ctx *c) : prev(t_prof) { t_prof = c ? &c->prof : nullptr; }
  ~ProfBind() { t_prof = prev; }
};
}  // namespace gf

struct gf_batch {
  gf_ctx *ctx = nullptr;
  uint64_t uid = 0;
  int n = 0;
  bool shared = false;
  std::vector<gf::StampDesc> h_desc;
  gf::StampDesc *d_desc = nullptr;
  int64_t n_pix = 0, n_pad = 0, n_psf = 0, n_par = 0, n_img = 0, n_jac = 0;
  int max_nc = 0, max_P = 0;
  // work lists
  std::vector<gf::Work> h_eval, h_pix, h_neq;   // h_neq: the units of stamps >= kNeqBigPix first
  int n_neq_big = 0;
  gf::Work *d_eval = nullptr, *d_pix = nullptr, *d_neq = nullptr;
  std::vector<int32_t> h_pix_first, h_neq_first, h_eval_first;   // first unit index per stamp (+ total)
  int32_t *d_pix_first = nullptr, *d_neq_first = nullptr, *d_eval_first = nullptr;
  // per-(stamp, component) constants of the current evaluation, rewritten by
  // every evaluation launch (calls on one batch are ordered on its context's
  // stream)
  gf::CompC *d_cc = nullptr;
  bool uniform = true;
  // observation groups (gf_batch_create_grouped): members of group g are
  // d_gmembers[d_gfirst[g] .. d_gfirst[g+1]); one group per stamp otherwise
  int n_groups = 0;
  std::vector<int32_t> h_gfirst, h_gmembers;
  int32_t *d_gfirst = nullptr, *d_gmembers = nullptr;
};

struct gf_psf {
  gf_ctx *ctx = nullptr;
  uint64_t uid = 0;
  const gf_batch *batch = nullptr;
  const float *d_taps = nullptr;
  std::vector<gf::PathDesc> h_path;
  gf::PathDesc *d_path = nullptr;
  std::vector<gf::FftPlan> h_plans;
  gf::FftPlan *d_plans = nullptr;
  float2 *d_tw = nullptr;      // twiddles of every plan, concatenated
  float2 *d_otf = nullptr;     // OTFs [L][L/2+1] per stamp (one if shared)
  int64_t n_otf = 0;
  int max_L = 0;
  int rmax = 18;               // largest plan radix class: 18, 24 or 32 (the FFT kernels are built for each)
  // FFT work lists: forward rows (padded rows), columns, inverse rows (output rows)
  std::vector<gf::Work> h_rows, h_cols, h_irows, h_arows, h_acols, h_airows;
  gf::Work *d_rows = nullptr, *d_cols = nullptr, *d_irows = nullptr;
  gf::Work *d_arows = nullptr, *d_acols = nullptr, *d_airows = nullptr;  // adjoint (correlation) lists
  std::vector<gf::Work> h_rows_n, h_cols_n, h_irows_n;                // narrow launch shape
  gf::Work *d_rows_n = nullptr, *d_cols_n = nullptr, *d_irows_n = nullptr;
  std::vector<int64_t> h_s1, h_s2;   // per-stamp offsets (complex) into the two spectra buffers, per channel
  int64_t n_s1 = 0, n_s2 = 0, n_s1a = 0, n_s2a = 0;
  int64_t *d_s1 = nullptr, *d_s2 = nullptr, *d_s1a = nullptr, *d_s2a = nullptr;
  std::vector<int64_t> h_s1a, h_s2a;
  // direct path tiles
  std::vector<gf::Work> h_direct, h_adirect;
  gf::Work *d_direct = nullptr, *d_adirect = nullptr;
  // chi^2 partial slots of the fused evaluations: an FFT stamp has one per
  // output row pair (from the inverse-row pass), a direct stamp one per
  // kPixChunk pixels (from the chi^2 kernel over h_pix_direct)
  std::vector<int32_t> h_c2_first;
  int32_t *d_c2_first = nullptr;
  int64_t n_c2 = 0;
  std::vector<gf::Work> h_pix_direct;
  gf::Work *d_pix_direct = nullptr;
  // one-workgroup FFT convolutions (sides up to kF2dMaxL): one entry per
  // stamp (unit = its bucket), grouped by bucket and side; the OTFs of these
  // stamps are stored row-major [L][L/2+1]
  std::vector<gf::Work> h_f2d;
  gf::Work *d_f2d = nullptr;
  int f2d_first[gf::kF2dBuckets + 1] = {};
  // multi-pass work units of the one-workgroup stamps (spectra offsets and a
  // bin-major OTF are kept for them too), used when few of a bucket's
  // stamps are still fitting: gf_fit_lm then moves them to the multi-pass
  // launches, which spread one stamp over many workgroups
  std::vector<gf::Work> h_rows_alt, h_cols_alt, h_irows_alt, h_rows_n_alt, h_cols_n_alt, h_irows_n_alt;
  gf::Work *d_rows_alt = nullptr, *d_cols_alt = nullptr, *d_irows_alt = nullptr;
  gf::Work *d_rows_n_alt = nullptr, *d_cols_n_alt = nullptr, *d_irows_n_alt = nullptr;
  // runs of the lists that LM fits restrict (built on the first fit)
  mutable std::vector<gf::ListRuns> lm_runs;
  int n_fft = 0, n_direct = 0, n_f2d = 0;
};

struct gf_line_batch {
  gf_ctx *ctx = nullptr;
  int n = 0;
  std::vector<gf::LineDesc> h_desc;
  gf::LineDesc *d_desc = nullptr;
  int64_t n_data = 0, n_lsf = 0, n_par = 0;
  bool has_nl[GF_LINE_MAX_LINES + 1] = {};
};

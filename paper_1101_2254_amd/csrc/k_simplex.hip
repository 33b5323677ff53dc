// k_simplex.hip -- downhill simplex (Nelder & Mead 1965) over a batch of
// stamps: the paper's other step-4 route besides Levenberg-Marquardt
// (Sec. 2), sharing steps 1-3 with it.
//
// Every stamp runs its own simplex state machine.  Each device iteration
// evaluates one candidate point per active stamp (steps 1-3 as usual) and
// then k_nm_step takes its chi^2 and emits the next candidate:
//   INIT k     vertex 0 = x0, vertex j+1 = x0 + step_j e_j, one per iteration
//   REFLECT    x_r = c + (c - x_w), c the centroid of the vertices but the worst
//   EXPAND     x_e = c + 2 (x_r - c)                  (if f_r < f_best)
//   CONTRACT   x_c = c + (x_r - c)/2 if f_r < f_w, else x_c = c + (x_w - c)/2
//   SHRINK k   x_i = x_b + (x_i - x_b)/2 for every i != b, evaluated in turn
// x_r replaces the worst vertex if f_best <= f_r < f_second-worst; x_e if
// f_e < f_r (else x_r); an outside contraction if f_c <= f_r, an inside one
// if f_c < f_w; otherwise the simplex shrinks.  Emitted points are clipped
// into [lo, hi].  Best, worst and second-worst are taken by (f, index): ties
// go to the lower index for the best and to the higher for the worst; NaN
// counts as +infinity.  At the start of each iteration a stamp stops when
// 2 (f_w - f_b) <= ftol (|f_w| + |f_b|) + 1e-300, or after max_iter
// iterations.
#include "gf_internal.h"
#include "twosum.h"

namespace gf {

enum { NM_INIT = 0, NM_REFLECT = 1, NM_EXPAND = 2, NM_CONTRACT = 3, NM_SHRINK = 4 };
enum { EMIT_VERTEX = 0, EMIT_REFLECT = 1, EMIT_EXPAND = 2, EMIT_CONTRACT = 3, EMIT_DONE = 4 };

struct NMState {
  int32_t phase, k, iters, nfev;
  int32_t active, status, reason, inside;
  int32_t b, w, sw, pad0;
  double f_r;
};

struct NMParams {
  int max_iter;
  double ftol;
  const double *lo, *hi;
};

constexpr int kNMV = kMaxP + 1;   // vertex slots per stamp

// X: [n][kNMV][kMaxP] vertices, F: [n][kNMV] values, XR: [n][kMaxP] the
// reflection point of the current iteration.
__global__ void k_nm_init(const StampDesc *__restrict__ desc, int n, const double *__restrict__ theta,
                          const double *__restrict__ step, NMParams prm, double *__restrict__ X,
                          double *__restrict__ theta_t, NMState *__restrict__ st, int *__restrict__ mask,
                          int *__restrict__ active_count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    const StampDesc d = desc[s];
    const int P = kNPC * d.ncomp + 1;
    double *xs = X + (int64_t)s * kNMV * kMaxP;
    for (int v = 0; v <= P; ++v)
      for (int q = 0; q < P; ++q) {
        double x = theta[d.par + q];
        if (v > 0 && q == v - 1) x += step ? step[d.par + q] : 0.0;
        if (prm.lo) x = fmax(x, prm.lo[d.par + q]);
        if (prm.hi) x = fmin(x, prm.hi[d.par + q]);
        xs[v * kMaxP + q] = x;
      }
    for (int q = 0; q < P; ++q) theta_t[d.par + q] = xs[q];
    NMState S{};
    S.phase = NM_INIT;
    S.active = 1;
    S.status = GF_ENOTCONV;
    S.reason = 5;
    st[s] = S;
    mask[s] = 1;
  }
  if (s == 0) *active_count = n;
}

// Best (lowest (f, index)), worst (highest, ties to the higher index) and
// second worst of F[0..P].
__device__ void nm_order(const double *fs, int P, int &b, int &w, int &sw) {
  b = 0;
  w = 0;
  for (int v = 1; v <= P; ++v) {
    if (fs[v] < fs[b]) b = v;
    if (fs[v] >= fs[w]) w = v;
  }
  sw = (w == 0) ? 1 : 0;
  for (int v = 0; v <= P; ++v)
    if (v != w && fs[v] >= fs[sw]) sw = v;
}

// One wave per stamp: lane 0 runs the state machine, lane q < P moves
// coordinate q of the vertices.
__global__ __launch_bounds__(64) void k_nm_step(const StampDesc *__restrict__ desc,
                                                const int32_t *__restrict__ pix_first,
                                                const float2 *__restrict__ part, NMParams prm,
                                                NMState *__restrict__ st, double *__restrict__ X,
                                                double *__restrict__ F, double *__restrict__ XR,
                                                double *__restrict__ theta_t, int *__restrict__ mask,
                                                double *__restrict__ trace, int trace_cap,
                                                int *__restrict__ active_count) {
  // store: -1 nothing, 0 x_t into X[w], 1 XR into X[w]; shrink: 0/1
  __shared__ int sh_store, sh_shrink, sh_emit;
  __shared__ NMState sS;
  const int s = blockIdx.x, lane = threadIdx.x;
  if (lane == 0) sS = st[s];
  __syncthreads();
  if (!sS.active) return;
  const StampDesc d = desc[s];
  const int P = kNPC * d.ncomp + 1;
  double *xs = X + (int64_t)s * kNMV * kMaxP;
  double *fs = F + (int64_t)s * kNMV;
  double *xr = XR + (int64_t)s * kMaxP;
  F2 r = {0.f, 0.f};
  for (int u = pix_first[s] + lane; u < pix_first[s + 1]; u += 64) {
    const float2 v = part[u];
    F2 x = {v.x, v.y};
    r = f2_add(r, x);
  }
  r = wave_sum(r);
  double ft = (double)r.hi + (double)r.lo;
  if (isnan(ft)) ft = INFINITY;
  const double xt = lane < P ? theta_t[d.par + lane] : 0.0;
  if (lane == 0) {
    NMState &S = sS;
    if (trace && S.nfev < trace_cap) trace[(int64_t)s * trace_cap + S.nfev] = ft;
    S.nfev += 1;
    int store = -1, shrink = 0, emit = EMIT_REFLECT;   // EMIT_REFLECT: start a new iteration
    if (S.phase == NM_INIT || S.phase == NM_SHRINK) {
      fs[S.k] = ft;                          // the candidate is vertex k itself
      int k = S.k + 1;
      if (S.phase == NM_SHRINK && k == S.b) ++k;
      if (k <= P) {
        S.k = k;
        emit = EMIT_VERTEX;
      }
    } else if (S.phase == NM_REFLECT) {
      if (ft < fs[S.b]) {
        S.f_r = ft;
        emit = EMIT_EXPAND;
      } else if (ft < fs[S.sw]) {
        store = 0;
        fs[S.w] = ft;
      } else {
        S.f_r = ft;
        S.inside = ft < fs[S.w] ? 0 : 1;
        emit = EMIT_CONTRACT;
      }
    } else if (S.phase == NM_EXPAND) {
      if (ft < S.f_r) {
        store = 0;
        fs[S.w] = ft;
      } else {
        store = 1;
        fs[S.w] = S.f_r;
      }
    } else {  // NM_CONTRACT
      if (S.inside ? ft < fs[S.w] : ft <= S.f_r) {
        store = 0;
        fs[S.w] = ft;
      } else {
        shrink = 1;
        S.phase = NM_SHRINK;
        S.k = (S.b == 0) ? 1 : 0;
        emit = EMIT_VERTEX;
      }
    }
    if (emit == EMIT_REFLECT) {
      int b, w, sw;
      nm_order(fs, P, b, w, sw);
      S.b = b;
      S.w = w;
      S.sw = sw;
      // the store above targets the old worst slot: it was written to fs
      // already, so order from the updated values
      const double fb = fs[b], fw = fs[w];
      if (2.0 * (fw - fb) <= prm.ftol * (fabs(fw) + fabs(fb)) + 1e-300) {
        S.active = 0;
        S.status = GF_OK;
        S.reason = 1;
        emit = EMIT_DONE;
      } else if (S.iters >= prm.max_iter) {
        S.active = 0;
        S.status = GF_ENOTCONV;
        S.reason = 5;
        emit = EMIT_DONE;
      } else {
        S.iters += 1;
        S.phase = NM_REFLECT;
      }
    } else if (emit == EMIT_EXPAND) {
      S.phase = NM_EXPAND;
    } else if (emit == EMIT_CONTRACT) {
      S.phase = NM_CONTRACT;
    }
    sh_store = store;
    sh_shrink = shrink;
    sh_emit = emit;
  }
  __syncthreads();
  const NMState S = sS;
  const int emit = sh_emit;
  // The store and the shrink use the worst/best of the iteration that made
  // the candidate; a new ordering (emit == REFLECT or DONE) was computed
  // after the value was stored, and the coordinates follow here.
  __shared__ int sh_wold;
  if (lane == 0) sh_wold = st[s].w;
  __syncthreads();
  if (lane < P) {
    const int wold = sh_wold;
    if (sh_store == 0) xs[wold * kMaxP + lane] = xt;
    if (sh_store == 1) xs[wold * kMaxP + lane] = xr[lane];
    if (sh_shrink) {
      const double xb = xs[S.b * kMaxP + lane];
      for (int v = 0; v <= P; ++v)
        if (v != S.b) xs[v * kMaxP + lane] = xb + 0.5 * (xs[v * kMaxP + lane] - xb);
    }
  }
  __syncthreads();
  if (lane < P) {
    double y;
    if (emit == EMIT_DONE) {
      y = xs[S.b * kMaxP + lane];   // the best vertex, returned to the caller
    } else if (emit == EMIT_VERTEX) {
      y = xs[S.k * kMaxP + lane];
    } else {
      double c = 0.0;
      for (int v = 0; v <= P; ++v)
        if (v != S.w) c += xs[v * kMaxP + lane];
      c /= (double)P;
      if (emit == EMIT_REFLECT) y = c + (c - xs[S.w * kMaxP + lane]);
      else if (emit == EMIT_EXPAND) y = c + 2.0 * (xr[lane] - c);
      else y = S.inside ? c + 0.5 * (xs[S.w * kMaxP + lane] - c) : c + 0.5 * (xr[lane] - c);
      if (prm.lo) y = fmax(y, prm.lo[d.par + lane]);
      if (prm.hi) y = fmin(y, prm.hi[d.par + lane]);
      if (emit == EMIT_REFLECT) xr[lane] = y;
    }
    theta_t[d.par + lane] = y;
  }
  __syncthreads();
  if (lane == 0) {
    st[s] = S;
    mask[s] = S.active;
    if (S.active) atomicAdd(active_count, 1);
  }
}

__global__ void k_nm_result(const StampDesc *__restrict__ desc, int n, const NMState *__restrict__ st,
                            const double *__restrict__ F, const double *__restrict__ X, double *__restrict__ theta,
                            gf_lm_result *__restrict__ res) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const NMState S = st[s];
  const StampDesc d = desc[s];
  const int P = kNPC * d.ncomp + 1;
  const double *fs = F + (int64_t)s * kNMV;
  const double *xs = X + (int64_t)s * kNMV * kMaxP;
  // best vertex of the final simplex (also for stamps stopped by the caller's cap)
  int b = 0;
  const int nv = S.phase == NM_INIT ? S.k : P + 1;
  for (int v = 1; v < nv; ++v)
    if (fs[v] < fs[b]) b = v;
  if (nv > 0) {
    for (int q = 0; q < P; ++q) theta[d.par + q] = xs[b * kMaxP + q];
  }
  gf_lm_result r;
  r.chi2 = nv > 0 ? fs[b] : INFINITY;
  r.lambda = 0.0;
  r.iters = S.iters;
  r.nfev = S.nfev;
  r.njev = 0;
  r.status = S.active ? GF_ENOTCONV : S.status;
  r.reason = S.active ? 5 : S.reason;
  r.pad = 0;
  res[s] = r;
}

hipError_t launch_nm_init(hipStream_t st, const gf_batch *b, const double *theta, const double *step,
                          const gf_simplex_opts *o, double *X, double *theta_t, void *S, int *mask, int *cnt) {
  NMParams prm{o->max_iter, o->ftol, o->lo, o->hi};
  hipLaunchKernelGGL(k_nm_init, dim3((b->n + 255) / 256), dim3(256), 0, st, b->d_desc, b->n, theta, step, prm, X,
                     theta_t, (NMState *)S, mask, cnt);
  return hipGetLastError();
}

hipError_t launch_nm_step(hipStream_t st, const gf_batch *b, const int32_t *first, const float2 *part,
                          const gf_simplex_opts *o, void *S,
                          double *X, double *F, double *XR, double *theta_t, int *mask, double *trace, int trace_cap,
                          int *cnt) {
  NMParams prm{o->max_iter, o->ftol, o->lo, o->hi};
  ProfScope ps(st, "k_nm_step");
  hipLaunchKernelGGL(k_nm_step, dim3(b->n), dim3(64), 0, st, b->d_desc, first, part, prm, (NMState *)S, X,
                     F, XR, theta_t, mask, trace, trace_cap, cnt);
  return hipGetLastError();
}

hipError_t launch_nm_result(hipStream_t st, const gf_batch *b, const void *S, const double *F, const double *X,
                            double *theta, gf_lm_result *res) {
  hipLaunchKernelGGL(k_nm_result, dim3((b->n + 255) / 256), dim3(256), 0, st, b->d_desc, b->n, (const NMState *)S, F,
                     X, theta, res);
  return hipGetLastError();
}

__global__ void k_nm_zero(int *__restrict__ c) { *c = 0; }

hipError_t launch_nm_zero(hipStream_t st, int *cnt) {
  hipLaunchKernelGGL(k_nm_zero, dim3(1), dim3(1), 0, st, cnt);
  return hipGetLastError();
}

size_t nm_state_bytes() { return sizeof(NMState); }

}  // namespace gf

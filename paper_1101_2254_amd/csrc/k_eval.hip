// k_eval.hip -- step 1 of the fitting loop (model evaluation on the pixel
// grid, a per-pixel transform: Barsdell et al., Sec. 2 step 1 and Sec. 3
// item 1) and its derivatives, for gfx950.
//
// Each workgroup of 256 threads (four wave64) owns 256 consecutive pixels of
// one stamp's padded grid, one pixel per thread, so every wave stores one
// contiguous 256-byte segment.  The work is arithmetic: per sub-sample and
// component one log2 and two exp2 (hardware v_log_f32 / v_exp_f32) plus about
// nine FMA-class operations; the output is 4 bytes per pixel.
//
// Sub-sample offsets relative to the centre are formed as
//     dx = (j - round(x0)) + ((s + 1/2)/S - 1/2 - (x0 - round(x0)))
// with the second bracket computed once per workgroup to one rounding, so
// that dx keeps full relative precision near the centre, where the Sersic
// cusp (R/Re)^(1/n) is steep, and is exactly zero when the centre sits on a
// sub-sample.
#include "gf_internal.h"
#include "comp.h"

namespace gf {

// One thread per (stamp, component): the constants every pixel of the
// component needs, computed once per launch instead of once per workgroup
// (the set-up costs about as many instructions as one wave's whole pixel
// loop at S = 5).
template <typename TT>
__global__ void k_comp_prep(const StampDesc *__restrict__ desc, int n, const TT *__restrict__ theta,
                            const float4 *__restrict__ bn_tab, int S, CompC *__restrict__ cc,
                            const int *__restrict__ mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = i / kMaxComp, k = i - s * kMaxComp;
  if (s >= n || (mask && !mask[s])) return;
  const StampDesc d = desc[s];
  if (k < d.ncomp) comp_setup<TT>(theta + d.par + kNPC * k, bn_tab, S, cc[i]);
}

// Start of an LM fit: the start point (read from start, or from theta when
// start is null) clipped into the box (written to theta and to the trial
// buffer) and its component constants, in one launch.
// Thread (stamp, k) clips the seven parameters of component k, and the sky
// for k = 0, then sets up component k from the clipped values.
__global__ void k_lm_start(const StampDesc *__restrict__ desc, int n, const double *start, double *theta,
                           const double *__restrict__ lo, const double *__restrict__ hi,
                           double *__restrict__ theta_t, const float4 *__restrict__ bn_tab, int S,
                           CompC *__restrict__ cc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = i / kMaxComp, k = i - s * kMaxComp;
  if (s >= n) return;
  const StampDesc d = desc[s];
  if (k >= d.ncomp) return;
  auto clip = [&](int64_t j) {
    double v = start ? start[j] : theta[j];
    if (lo && v < lo[j]) v = lo[j];
    if (hi && v > hi[j]) v = hi[j];
    theta[j] = v;
    theta_t[j] = v;
    return v;
  };
  double t[kNPC];
#pragma unroll
  for (int q = 0; q < kNPC; ++q) t[q] = clip(d.par + kNPC * k + q);
  if (k == 0) (void)clip(d.par + kNPC * d.ncomp);
  comp_setup<double>(t, bn_tab, S, cc[i]);
}

// ----------------------------------------------------------------- values
// R^2 = x'^2 + (y'/q)^2 with y'/q formed directly from cos phi / q and
// sin phi / q (one multiply fewer per sub-sample than scaling y'^2).
template <int S>
__global__ __launch_bounds__(kThreads) void k_eval(const StampDesc *__restrict__ desc, const Work *__restrict__ work,
                                                   const CompC *__restrict__ cc, float *__restrict__ out,
                                                   const int *__restrict__ mask) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  cc += (int64_t)s * kMaxComp;
  const int npad = d.Mh * d.Mw;
  const int p = w.unit * kEvalTile + (int)threadIdx.x;
  if (p >= npad) return;
  const int pi = p / d.Mw, pj = p - pi * d.Mw;
  const int c0 = (d.K - 1) >> 1;
  const int i = pi - c0, j = pj - c0;
  float acc = 0.0f;
  for (int k = 0; k < d.ncomp; ++k) {
    const CompC C = cc[k];
    const float jx = (float)(j - C.ix), iy = (float)(i - C.iy);
    const float peak = C.lie + C.b1;
    float ox[S];
#pragma unroll
    for (int a = 0; a < S; ++a) ox[a] = jx + C.ox[a];
#pragma unroll
    for (int b = 0; b < S; ++b) {
      const float dy = iy + C.oy[b];
      const float dysn = dy * C.sn, dycq = dy * C.cq;
#pragma unroll
      for (int a = 0; a < S; ++a) {
        const float dx = ox[a];
        const float xp = fmaf(dx, C.cs, dysn);
        const float yq = fmaf(-dx, C.sq, dycq);
        const float r2 = fmaf(yq, yq, xp * xp);
        const float t = fast_exp2(fmaf(fast_log2(r2), C.a1, C.a0));
        acc += fast_exp2(fmaf(-C.b1, t, peak));
      }
    }
  }
  out[d.pad + p] = acc * (1.0f / (float)(S * S));
}

// -------------------------------------------------------------- derivatives
// Point derivatives of one component at offset (dx, dy) from its centre, in
// parameter order [x0, y0, Ie, Re, n, q, phi]; the Ie slot holds I/Ie (the
// model is linear in Ie).  With u = R/Re, t = u^(1/n), E = b_n t:
// dI/dRe = I E/(n Re),  dI/dn = I (b'_n (1-t) + E ln u/n^2),
// dI/d(R^2) = -I E/(2 n R^2).  At R = 0 exactly the 1/R^2 and ln u terms are 0.
// The rotation, axis-ratio and n factors are constants of the component, so
// each sub-sample only adds to eight sums (w = -2 dI/d(R^2), x' and y' the
// rotated offsets, y'' = y'/q^2):
//   U = sum w x', V = sum w y'', W5 = sum w y'' y', W6 = sum w x' y',
//   sum I/Ie, sum I E, A4 = sum I (1-t), B4 = sum I E log2 t,
// and grad_finish turns them into the seven derivatives once per pixel.
struct GradAcc {
  float U = 0.f, V = 0.f, W5 = 0.f, W6 = 0.f, Js = 0.f, IEs = 0.f, A4 = 0.f, B4 = 0.f;
};

__device__ __forceinline__ void grad_acc(const CompC &C, float dx, float dy, GradAcc &a) {
  const float xp = fmaf(dx, C.cs, dy * C.sn);
  const float yp = fmaf(-dx, C.sn, dy * C.cs);
  const float yi = C.iq2 * yp;
  const float r2 = fmaf(yi, yp, xp * xp);
  const float l2 = fast_log2(r2);
  const float lt = fmaf(l2, C.a1, C.a0);               // log2 t
  const float t = fast_exp2(lt);
  const float omt = 1.0f - t;
  const float J = fast_exp2(C.b1 * omt);               // I / Ie
  const float I = J * C.ie;
  const float IE = I * (C.bn * t);
  const bool nz = r2 > 0.0f;
  const float w = nz ? (IE * C.inv_n) * __builtin_amdgcn_rcpf(r2) : 0.0f;   // -2 dI / d(R^2)
  const float u = w * xp, v = w * yi;
  a.U += u;
  a.V += v;
  a.W5 = fmaf(v, yp, a.W5);
  a.W6 = fmaf(u, yp, a.W6);
  a.Js += J;
  a.IEs += IE;
  a.A4 = fmaf(I, omt, a.A4);
  a.B4 = fmaf(IE, nz ? lt : 0.0f, a.B4);
}

// d x'/d x0 = -cos, d y'/d x0 = sin, ... applied to the sums; ln u / n^2 =
// log2(t) ln 2 / n.
__device__ __forceinline__ void grad_finish(const CompC &C, const GradAcc &a, float *g) {
  g[0] = fmaf(C.cs, a.U, -C.sn * a.V);
  g[1] = fmaf(C.sn, a.U, C.cs * a.V);
  g[2] = a.Js;
  g[3] = a.IEs * (C.inv_n * C.inv_re);
  g[4] = fmaf(C.dbn, a.A4, a.B4 * (0.69314718055994531f * C.inv_n));
  g[5] = a.W5 * C.inv_q;
  g[6] = -a.W6 * (1.0f - C.iq2);
}

// Writes 7 * ncomp channels per stamp on the padded grid: channel 7k + p is
// the sub-sample mean of d I_k / d theta_{k,p} (p = 2 holds I_k / Ie_k).
// Layout: out[jac_pad_off(s) + ch * Mh*Mw + pixel] with jac_pad_off = 7 * pad
// offset scaled by the channel count of the batch (chan_stride channels per
// stamp).
template <int S>
__global__ __launch_bounds__(kThreads) void k_eval_jac(const StampDesc *__restrict__ desc,
                                                       const Work *__restrict__ work, const CompC *__restrict__ cc,
                                                       float *__restrict__ out, int chan_stride,
                                                       const int *__restrict__ mask) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  cc += (int64_t)s * kMaxComp;
  const int npad = d.Mh * d.Mw;
  const int p = w.unit * kEvalTile + (int)threadIdx.x;
  if (p >= npad) return;
  const int pi = p / d.Mw, pj = p - pi * d.Mw;
  const int c0 = (d.K - 1) >> 1;
  const int i = pi - c0, j = pj - c0;
  float *o = out + d.pad * (int64_t)chan_stride + p;
  for (int k = 0; k < d.ncomp; ++k) {
    const CompC C = cc[k];
    const float jx = (float)(j - C.ix), iy = (float)(i - C.iy);
    GradAcc acc;
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      const float dy = iy + cc[k].oy[b];
#pragma unroll
      for (int a = 0; a < S; ++a) grad_acc(C, jx + C.ox[a], dy, acc);
    }
    float g[kNPC];
    grad_finish(C, acc, g);
    const bool no_ie = skip_ie(mask, s, kNPC * k + 2);
#pragma unroll
    for (int q = 0; q < kNPC; ++q)
      if (!(q == 2 && no_ie)) o[(int64_t)(kNPC * k + q) * npad] = g[q] * (1.0f / (float)(S * S));
  }
}

// Adjoint contraction on the padded grid: for every stamp,
//   part[chunk][p] = sum over the chunk's pixels of adj[pixel] * dM/dtheta_p
// (component parameters only; the sky term is added by the caller).
// adj holds one padded grid per stamp at desc.pad.
template <int S>
__global__ __launch_bounds__(kThreads) void k_adjoint_contract(const StampDesc *__restrict__ desc,
                                                               const Work *__restrict__ work,
                                                               const CompC *__restrict__ cc,
                                                               const float *__restrict__ adj,
                                                               const int32_t *__restrict__ first,
                                                               float *__restrict__ part) {
  __shared__ float red[kThreads / 64][kMaxP];
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  const StampDesc d = desc[s];
  cc += (int64_t)s * kMaxComp;
  const int npad = d.Mh * d.Mw;
  const int p = w.unit * kEvalTile + (int)threadIdx.x;
  const int nq = kNPC * d.ncomp;
  float acc[kMaxP - 1];
#pragma unroll
  for (int q = 0; q < kMaxP - 1; ++q) acc[q] = 0.0f;
  if (p < npad) {
    const int pi = p / d.Mw, pj = p - pi * d.Mw;
    const int c0 = (d.K - 1) >> 1;
    const int i = pi - c0, j = pj - c0;
    const float a = adj[d.pad + p] * (1.0f / (float)(S * S));
    for (int k = 0; k < d.ncomp; ++k) {
      const CompC C = cc[k];
      const float jx = (float)(j - C.ix), iy = (float)(i - C.iy);
      GradAcc ga;
#pragma unroll 1
      for (int b = 0; b < S; ++b) {
        const float dy = iy + cc[k].oy[b];
#pragma unroll
        for (int aa = 0; aa < S; ++aa) grad_acc(C, jx + C.ox[aa], dy, ga);
      }
      float g[kNPC];
      grad_finish(C, ga, g);
      // Ie slot: dI/dIe = I/Ie
#pragma unroll
      for (int q = 0; q < kNPC; ++q) {
#pragma unroll
        for (int kk = 0; kk < kMaxComp; ++kk)
          if (kk == k) acc[kNPC * kk + q] = a * g[q];
      }
    }
  }
  // block reduction in a fixed order: wave shuffles, then the four waves
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kMaxP - 1; ++q) {
    float v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nq) {
    float v = 0.0f;
#pragma unroll
    for (int ww = 0; ww < kThreads / 64; ++ww) v += red[ww][threadIdx.x];
    part[(int64_t)(first[s] + w.unit) * (kMaxP - 1) + threadIdx.x] = v;   // the unit's own slot
  }
}

// ----------------------------------------------------------------- launchers
template <typename TT>
static hipError_t launch_prep(hipStream_t st, const gf_batch *b, const TT *theta, int S, const float4 *bn,
                              const int *mask, CompC *cc) {
  const int nt = b->n * kMaxComp;
  hipLaunchKernelGGL((k_comp_prep<TT>), dim3((nt + 63) / 64), dim3(64), 0, st, b->d_desc, b->n, theta, bn, S, cc,
                     mask);
  return hipGetLastError();
}

template <typename TT>
static hipError_t launch_eval_t(hipStream_t st, const gf_batch *b, const TT *theta, int S, const float4 *bn,
                                float *out, const int *mask, const WorkView *v, CompC *cc, bool prep) {
  const Work *lst = v && v->eval ? v->eval : b->d_eval;
  dim3 grid((unsigned)(v && v->eval ? v->n_eval : (int)b->h_eval.size())), block(kThreads);
  if (grid.x == 0) return hipSuccess;
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return hipErrorInvalidValue;
  if (!cc) cc = b->d_cc;
  if (prep) {
    hipError_t e = launch_prep<TT>(st, b, theta, S, bn, mask, cc);
    if (e != hipSuccess) return e;
  }
  ProfScope ps(st, "k_eval");
  switch (S) {
#define GF_EVAL_CASE(SS)                                                                        \
  case SS:                                                                                      \
    hipLaunchKernelGGL((k_eval<SS>), grid, block, 0, st, b->d_desc, lst, cc, out, mask);       \
    break;
    GF_EVAL_CASE(1) GF_EVAL_CASE(2) GF_EVAL_CASE(3) GF_EVAL_CASE(4)
    GF_EVAL_CASE(5) GF_EVAL_CASE(6) GF_EVAL_CASE(7) GF_EVAL_CASE(8)
#undef GF_EVAL_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_eval(hipStream_t st, const gf_batch *b, const float *theta, int S, const float4 *bn, float *out,
                       const int *mask) {
  return launch_eval_t<float>(st, b, theta, S, bn, out, mask, nullptr, nullptr, true);
}

// cc: where the component constants live (null: the batch's buffer); prep:
// compute them from theta first (false: the caller keeps them current).
hipError_t launch_lm_start(hipStream_t st, const gf_batch *b, const double *start, double *theta, const double *lo,
                           const double *hi, double *theta_t, int S, const float4 *bn, CompC *cc) {
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return hipErrorInvalidValue;
  const int nt = b->n * kMaxComp;
  hipLaunchKernelGGL(k_lm_start, dim3((nt + 63) / 64), dim3(64), 0, st, b->d_desc, b->n, start, theta, lo, hi, theta_t, bn,
                     S, cc);
  return hipGetLastError();
}

hipError_t launch_eval_d(hipStream_t st, const gf_batch *b, const double *theta, int S, const float4 *bn,
                         float *out, const int *mask, const WorkView *v, CompC *cc, bool prep) {
  return launch_eval_t<double>(st, b, theta, S, bn, out, mask, v, cc, prep);
}

template <typename TT>
static hipError_t launch_eval_jac_t(hipStream_t st, const gf_batch *b, const TT *theta, int S, const float4 *bn,
                                    float *out, int chan_stride, const int *mask, const WorkView *v, CompC *cc,
                                    bool prep) {
  const Work *lst = v && v->eval ? v->eval : b->d_eval;
  dim3 grid((unsigned)(v && v->eval ? v->n_eval : (int)b->h_eval.size())), block(kThreads);
  if (grid.x == 0) return hipSuccess;
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return hipErrorInvalidValue;
  if (!cc) cc = b->d_cc;
  if (prep) {
    hipError_t e = launch_prep<TT>(st, b, theta, S, bn, mask, cc);
    if (e != hipSuccess) return e;
  }
  ProfScope ps(st, "k_eval_jac");
  switch (S) {
#define GF_EVALJ_CASE(SS)                                                                                  \
  case SS:                                                                                                 \
    hipLaunchKernelGGL((k_eval_jac<SS>), grid, block, 0, st, b->d_desc, lst, cc, out, chan_stride, mask);     \
    break;
    GF_EVALJ_CASE(1) GF_EVALJ_CASE(2) GF_EVALJ_CASE(3) GF_EVALJ_CASE(4)
    GF_EVALJ_CASE(5) GF_EVALJ_CASE(6) GF_EVALJ_CASE(7) GF_EVALJ_CASE(8)
#undef GF_EVALJ_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_eval_jac(hipStream_t st, const gf_batch *b, const float *theta, int S, const float4 *bn,
                           float *out, int chan_stride, const int *mask) {
  return launch_eval_jac_t<float>(st, b, theta, S, bn, out, chan_stride, mask, nullptr, nullptr, true);
}

hipError_t launch_eval_jac_d(hipStream_t st, const gf_batch *b, const double *theta, int S, const float4 *bn,
                             float *out, int chan_stride, const int *mask, const WorkView *v, CompC *cc,
                             bool prep) {
  return launch_eval_jac_t<double>(st, b, theta, S, bn, out, chan_stride, mask, v, cc, prep);
}

hipError_t launch_adjoint_contract(hipStream_t st, const gf_batch *b, const float *theta, int S, const float4 *bn,
                                   const float *adj, float *part) {
  dim3 grid((unsigned)b->h_eval.size()), block(kThreads);
  if (grid.x == 0) return hipSuccess;
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return hipErrorInvalidValue;
  hipError_t e = launch_prep<float>(st, b, theta, S, bn, nullptr, b->d_cc);
  if (e != hipSuccess) return e;
  ProfScope ps(st, "k_adjoint_contract");
  switch (S) {
#define GF_ADJ_CASE(SS)                                                                                      \
  case SS:                                                                                                   \
    hipLaunchKernelGGL((k_adjoint_contract<SS>), grid, block, 0, st, b->d_desc, b->d_eval, b->d_cc, adj,         \
                       b->d_eval_first, part);                                                               \
    break;
    GF_ADJ_CASE(1) GF_ADJ_CASE(2) GF_ADJ_CASE(3) GF_ADJ_CASE(4)
    GF_ADJ_CASE(5) GF_ADJ_CASE(6) GF_ADJ_CASE(7) GF_ADJ_CASE(8)
#undef GF_ADJ_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gf

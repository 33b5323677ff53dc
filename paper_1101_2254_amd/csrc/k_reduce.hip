// k_reduce.hip -- step 3 of the fitting loop (comparison of model and
// observation as the sum of squared differences: a transform followed by a
// reduce, Barsdell et al., Sec. 3 item 3) and the reductions behind the
// Levenberg-Marquardt update (steps 4-5), for gfx950.
//
// Sums are FP32 with error-free transformations: each thread keeps a (hi, lo)
// pair updated by TwoSum (Knuth), pairs are combined through wave64 shuffles
// and then across the workgroup's four waves in a fixed order, and the last
// workgroup of a stamp to finish (found with a per-stamp counter that resets
// itself) adds the workgroup partials in index order.  Nothing depends on the
// order in which workgroups run, so results are bitwise reproducible.
#include "gf_internal.h"

namespace gf {

struct F2 {
  float hi, lo;
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  F2 r;
  r.hi = s + e;
  r.lo = e - (r.hi - s);
  return r;
}

__device__ __forceinline__ F2 f2_add1(F2 a, float v) {
  float s, e;
  two_sum(a.hi, v, s, e);
  F2 r;
  r.hi = s;
  r.lo = a.lo + e;
  return r;
}

__device__ __forceinline__ F2 wave_sum(F2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    F2 o;
    o.hi = __shfl_xor(v.hi, off, 64);
    o.lo = __shfl_xor(v.lo, off, 64);
    v = f2_add(v, o);
  }
  return v;
}

// Workgroup sum of a pair; the result is valid in thread 0.
__device__ F2 block_sum(F2 v) {
  __shared__ F2 red[kThreads / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  F2 r = {0.f, 0.f};
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) r = f2_add(r, red[i]);
  }
  return r;
}

template <typename TT>
__device__ __forceinline__ float sky_of(const TT *theta, const StampDesc &d) {
  return (float)theta[d.par + kNPC * d.ncomp];
}

// ------------------------------------------------------------------ chi^2
// r = sqrt(w) (d - m - sky); chi2[s] = (hi, lo) of sum r^2.
template <typename TT>
__global__ __launch_bounds__(kThreads) void k_chi2(const StampDesc *__restrict__ desc, const Work *__restrict__ work,
                                                   const int32_t *__restrict__ first, const float *__restrict__ model,
                                                   const TT *__restrict__ theta, const float *__restrict__ data,
                                                   const float *__restrict__ weight, float *__restrict__ resid,
                                                   float2 *__restrict__ part, unsigned int *__restrict__ counters,
                                                   float2 *__restrict__ chi2, const int *__restrict__ mask) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  const float sky = sky_of(theta, d);
  const int npix = d.H * d.W;
  const int p0 = w.unit * kPixChunk;
  F2 acc = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = p0 + k * kThreads + (int)threadIdx.x;
    if (p < npix) {
      const float wt = weight[d.img + p];
      const float r = sqrtf(wt) * (data[d.img + p] - (model[d.pix + p] + sky));
      if (resid) resid[d.pix + p] = r;
      acc = f2_add1(acc, r * r);
    }
  }
  const F2 tot = block_sum(acc);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = make_float2(tot.hi, tot.lo);
    __threadfence();
    const unsigned int n_units = (unsigned)(first[s + 1] - first[s]);
    const unsigned int prev = atomicAdd(&counters[s], 1u);
    if (prev == n_units - 1) {
      __threadfence();
      F2 r = {0.f, 0.f};
      for (int u = first[s]; u < first[s + 1]; ++u) {
        const float2 v = part[u];
        F2 t = {v.x, v.y};
        r = f2_add(r, t);
      }
      chi2[s] = make_float2(r.hi, r.lo);
      counters[s] = 0u;
    }
  }
}

hipError_t launch_chi2(hipStream_t st, const gf_batch *b, const float *model, const void *theta, bool theta_f64,
                       const float *data, const float *weight, float *resid, float2 *part, unsigned int *counters,
                       float2 *chi2, const int *mask) {
  dim3 grid((unsigned)b->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  if (theta_f64)
    hipLaunchKernelGGL((k_chi2<double>), grid, blk, 0, st, b->d_desc, b->d_pix, b->d_pix_first, model,
                       (const double *)theta, data, weight, resid, part, counters, chi2, mask);
  else
    hipLaunchKernelGGL((k_chi2<float>), grid, blk, 0, st, b->d_desc, b->d_pix, b->d_pix_first, model,
                       (const float *)theta, data, weight, resid, part, counters, chi2, mask);
  return hipGetLastError();
}

// ------------------------------------------------- adjoint helpers
// c = scale * cot * (weight ? sqrt(weight) : 1) on the stamp grid, plus the
// per-chunk sums of c (the sky derivative of the contraction).
__global__ __launch_bounds__(kThreads) void k_cot_prep(const StampDesc *__restrict__ desc,
                                                       const Work *__restrict__ work, const float *__restrict__ cot,
                                                       const float *__restrict__ weight, float scale,
                                                       float *__restrict__ c, float2 *__restrict__ part) {
  const Work w = work[blockIdx.x];
  const StampDesc d = desc[w.stamp];
  const int npix = d.H * d.W;
  const int p0 = w.unit * kPixChunk;
  F2 acc = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = p0 + k * kThreads + (int)threadIdx.x;
    if (p < npix) {
      float v = scale * cot[d.pix + p];
      if (weight) v *= sqrtf(weight[d.img + p]);
      c[d.pix + p] = v;
      acc = f2_add1(acc, v);
    }
  }
  const F2 tot = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(tot.hi, tot.lo);
}

// out[par + q] = sum of contraction partials (component parameters) and
// out[par + P-1] = sum of the c partials (sky).  One thread per stamp.
__global__ void k_adjoint_final(const StampDesc *__restrict__ desc, int n, const int32_t *__restrict__ eval_first,
                                const float *__restrict__ cpart, const int32_t *__restrict__ pix_first,
                                const float2 *__restrict__ spart, float *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const StampDesc d = desc[s];
  const int nq = kNPC * d.ncomp;
  for (int q = 0; q < nq; ++q) {
    F2 r = {0.f, 0.f};
    for (int u = eval_first[s]; u < eval_first[s + 1]; ++u) {
      F2 t = {cpart[(int64_t)u * (kMaxP - 1) + q], 0.f};
      r = f2_add(r, t);
    }
    out[d.par + q] = r.hi + r.lo;
  }
  F2 r = {0.f, 0.f};
  for (int u = pix_first[s]; u < pix_first[s + 1]; ++u) {
    F2 t = {spart[u].x, spart[u].y};
    r = f2_add(r, t);
  }
  out[d.par + nq] = r.hi + r.lo;
}

hipError_t launch_cot_prep(hipStream_t st, const gf_batch *b, const float *cot, const float *weight, float scale,
                           float *c, float2 *spart) {
  dim3 grid((unsigned)b->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cot_prep, grid, blk, 0, st, b->d_desc, b->d_pix, cot, weight, scale, c, spart);
  return hipGetLastError();
}

hipError_t launch_adjoint_final(hipStream_t st, const gf_batch *b, const int32_t *d_eval_first, const float *cpart,
                                const float2 *spart, float *out) {
  const int nb = (b->n + 127) / 128;
  hipLaunchKernelGGL(k_adjoint_final, dim3(nb), dim3(128), 0, st, b->d_desc, b->n, d_eval_first, cpart,
                     b->d_pix_first, spart, out);
  return hipGetLastError();
}

// Full Jacobian images: out[jac + p*H*W + i] = jc[pix*nchan + p*H*W + i] for
// component parameters, and 1 for the sky.  One workgroup per pixel chunk.
__global__ __launch_bounds__(kThreads) void k_jac_assemble(const StampDesc *__restrict__ desc,
                                                           const Work *__restrict__ work,
                                                           const float *__restrict__ jc, int nchan,
                                                           float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const StampDesc d = desc[w.stamp];
  const int npix = d.H * d.W;
  const int p0 = w.unit * kPixChunk;
  const int nq = kNPC * d.ncomp;
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = p0 + k * kThreads + (int)threadIdx.x;
    if (p >= npix) break;
    for (int q = 0; q < nq; ++q)
      out[d.jac + (int64_t)q * npix + p] = jc[d.pix * (int64_t)nchan + (int64_t)q * npix + p];
    out[d.jac + (int64_t)nq * npix + p] = 1.0f;
  }
}

hipError_t launch_jac_assemble(hipStream_t st, const gf_batch *b, const float *jc, int nchan, float *out) {
  dim3 grid((unsigned)b->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  hipLaunchKernelGGL(k_jac_assemble, grid, blk, 0, st, b->d_desc, b->d_pix, jc, nchan, out);
  return hipGetLastError();
}

// m += sky (the model image of step 1-2 plus the constant sky).
__global__ __launch_bounds__(kThreads) void k_add_sky(const StampDesc *__restrict__ desc,
                                                      const Work *__restrict__ work, const float *__restrict__ theta,
                                                      float *__restrict__ m) {
  const Work w = work[blockIdx.x];
  const StampDesc d = desc[w.stamp];
  const int npix = d.H * d.W;
  const float sky = theta[d.par + kNPC * d.ncomp];
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = w.unit * kPixChunk + k * kThreads + (int)threadIdx.x;
    if (p < npix) m[d.pix + p] += sky;
  }
}

hipError_t launch_add_sky(hipStream_t st, const gf_batch *b, const float *theta, float *m) {
  dim3 grid((unsigned)b->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_sky, grid, blk, 0, st, b->d_desc, b->d_pix, theta, m);
  return hipGetLastError();
}

// --------------------------------------------------- normal equations
// For the stamps flagged in mask, per workgroup chunk of pixels:
//   A_pq = sum w j_p j_q (q <= p), g_p = sum w j_p r, chi2 = sum w r^2,
// with j the Jacobian row (convolved channels, Ie channels hold I/Ie; the
// sky column is 1) and r = d - m, m = sky + sum_k Ie_k * chan(Ie_k).
// jc: stamp s, channel ch at pix * nchan + ch * H*W (nchan = 7 * the
// largest component count of the batch).
template <int NC>
__global__ __launch_bounds__(kThreads) void k_normal_eq(const StampDesc *__restrict__ desc,
                                                        const Work *__restrict__ work, const float *__restrict__ jc,
                                                        const double *__restrict__ theta,
                                                        const float *__restrict__ data,
                                                        const float *__restrict__ weight, float *__restrict__ part,
                                                        int nacc_stride, int nchan, const int *__restrict__ mask) {
  constexpr int P = kNPC * NC + 1;
  constexpr int NA = P * (P + 1) / 2 + P + 1;
  __shared__ float red[kThreads / 64][NA];
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  if (d.ncomp != NC) return;
  const int npix = d.H * d.W;
  const int64_t plane = npix;
  const float *J = jc + d.pix * (int64_t)nchan;
  float ie[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) ie[k] = (float)theta[d.par + kNPC * k + 2];
  const float sky = (float)theta[d.par + kNPC * NC];
  float acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = 0.0f;
  const int p0 = w.unit * kNeqChunk;
#pragma unroll 1
  for (int k = 0; k < kNeqChunk / kThreads; ++k) {
    const int p = p0 + k * kThreads + (int)threadIdx.x;
    if (p >= npix) break;
    float j[P];
#pragma unroll
    for (int q = 0; q < P - 1; ++q) j[q] = J[q * plane + p];
    j[P - 1] = 1.0f;
    float m = sky;
#pragma unroll
    for (int c = 0; c < NC; ++c) m = fmaf(ie[c], j[kNPC * c + 2], m);
    const float wt = weight[d.img + p];
    const float r = data[d.img + p] - m;
    const float wr = wt * r;
    int a = 0;
#pragma unroll
    for (int p1 = 0; p1 < P; ++p1) {
      const float wj = wt * j[p1];
#pragma unroll
      for (int p2 = 0; p2 <= p1; ++p2) {
        acc[a] = fmaf(wj, j[p2], acc[a]);
        ++a;
      }
    }
#pragma unroll
    for (int p1 = 0; p1 < P; ++p1) {
      acc[a] = fmaf(wr, j[p1], acc[a]);
      ++a;
    }
    acc[a] = fmaf(wr, r, acc[a]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    float v = acc[a];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wv][a] = v;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < NA; a += blockDim.x) {
    float v = 0.0f;
#pragma unroll
    for (int ww = 0; ww < kThreads / 64; ++ww) v += red[ww][a];
    part[(int64_t)blockIdx.x * nacc_stride + a] = v;
  }
}

hipError_t launch_normal_eq(hipStream_t st, const gf_batch *b, const float *jc, const double *theta,
                            const float *data, const float *weight, float *part, int nacc_stride, int nchan,
                            const int *mask) {
  dim3 grid((unsigned)b->h_neq.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  bool has1 = false, has2 = false;
  for (const auto &d : b->h_desc) {
    has1 |= d.ncomp == 1;
    has2 |= d.ncomp == 2;
  }
  if (has1)
    hipLaunchKernelGGL((k_normal_eq<1>), grid, blk, 0, st, b->d_desc, b->d_neq, jc, theta, data, weight, part,
                       nacc_stride, nchan, mask);
  if (has2)
    hipLaunchKernelGGL((k_normal_eq<2>), grid, blk, 0, st, b->d_desc, b->d_neq, jc, theta, data, weight, part,
                       nacc_stride, nchan, mask);
  return hipGetLastError();
}

// ------------------------------------------------------------- LM kernels
struct LMParams {
  int32_t max_iter;
  double lambda_up, lambda_down, lambda_max, ftol, xtol;
  const double *lo, *hi;
  const uint8_t *free_mask;
};

// Start: chi2 of the (clipped) start point is in chi2t.
__global__ void k_lm_init(const StampDesc *__restrict__ desc, int n, double lambda0, const float2 *__restrict__ chi2t,
                          LMState *__restrict__ st, int *__restrict__ mjac, int *__restrict__ mtrial,
                          int *__restrict__ active_count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    LMState S;
    S.lambda = lambda0;
    S.chi2 = (double)chi2t[s].x + (double)chi2t[s].y;
    S.chi2_trial = S.chi2;
    S.iters = 0;
    S.nfev = 1;
    S.njev = 0;
    S.status = GF_ENOTCONV;
    S.reason = 5;
    S.active = 1;
    S.need_jac = 1;
    S.trial = 0;
    if (S.chi2 == 0.0) {
      S.status = GF_OK;
      S.reason = 3;
      S.active = 0;
    }
    st[s] = S;
    mjac[s] = S.active;
    mtrial[s] = 0;
  }
  if (s == 0) *active_count = n;
}

// Clip the start point into the box: theta_t = clip(theta).
__global__ void k_lm_clip(int64_t n_par, double *__restrict__ theta, const double *__restrict__ lo,
                          const double *__restrict__ hi, double *__restrict__ theta_t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_par) return;
  double v = theta[i];
  if (lo && v < lo[i]) v = lo[i];
  if (hi && v > hi[i]) v = hi[i];
  theta[i] = v;
  theta_t[i] = v;
}

// One wave64 per stamp: form A, g (FP64 sums of the workgroup partials) when
// the Jacobian is new, damp, factor by Cholesky, solve, write the clipped
// trial point.
__global__ __launch_bounds__(64) void k_lm_solve(const StampDesc *__restrict__ desc,
                                                 const int32_t *__restrict__ neq_first,
                                                 const float *__restrict__ part, int nacc_stride,
                                                 LMParams prm, LMState *__restrict__ st,
                                                 double *__restrict__ Ag /* per stamp kMaxP*kMaxP + kMaxP */,
                                                 const double *__restrict__ theta, double *__restrict__ theta_t,
                                                 int *__restrict__ mjac, int *__restrict__ mtrial) {
  __shared__ double A[kMaxP * kMaxP];
  __shared__ double g[kMaxP];
  __shared__ double Lm[kMaxP * kMaxP];
  __shared__ double y[kMaxP];
  __shared__ int idx[kMaxP];
  __shared__ int nf_s, ok_s;
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  LMState S = st[s];
  if (!S.active) return;
  const StampDesc d = desc[s];
  const int P = kNPC * d.ncomp + 1;
  double *Ags = Ag + (int64_t)s * (kMaxP * kMaxP + kMaxP);
  if (S.need_jac) {
    // accumulator order: lower triangle row-major (p1 >= p2), then g, then chi2
    const int NA = P * (P + 1) / 2 + P + 1;
    for (int a = lane; a < NA - 1; a += 64) {
      double v = 0.0;
      for (int u = neq_first[s]; u < neq_first[s + 1]; ++u) v += (double)part[(int64_t)u * nacc_stride + a];
      if (a < P * (P + 1) / 2) {
        int p1 = 0;
        while ((p1 + 1) * (p1 + 2) / 2 <= a) ++p1;
        const int p2 = a - p1 * (p1 + 1) / 2;
        Ags[p1 * kMaxP + p2] = v;
        Ags[p2 * kMaxP + p1] = v;
      } else {
        Ags[kMaxP * kMaxP + (a - P * (P + 1) / 2)] = v;
      }
    }
    __syncthreads();
  }
  if (lane == 0) {
    int nf = 0;
    for (int p = 0; p < P; ++p)
      if (!prm.free_mask || prm.free_mask[d.par + p]) idx[nf++] = p;
    nf_s = nf;
  }
  __syncthreads();
  const int nf = nf_s;
  for (int e = lane; e < nf * nf; e += 64) {
    const int a = e / nf, b = e - a * nf;
    A[e] = Ags[idx[a] * kMaxP + idx[b]];
  }
  for (int a = lane; a < nf; a += 64) g[a] = Ags[kMaxP * kMaxP + idx[a]];
  __syncthreads();
  if (lane == 0) {
    double dmax = 0.0;
    for (int a = 0; a < nf; ++a) dmax = fmax(dmax, A[a * nf + a]);
    for (int a = 0; a < nf; ++a) {
      const double da = fmax(A[a * nf + a], 1e-12 * dmax);
      A[a * nf + a] += S.lambda * da;
    }
    ok_s = 1;
  }
  __syncthreads();
  // Cholesky A = L L^T, column by column; rows of a column in parallel.
  for (int j = 0; j < nf; ++j) {
    if (lane == 0) {
      double sj = A[j * nf + j];
      for (int k = 0; k < j; ++k) sj -= Lm[j * nf + k] * Lm[j * nf + k];
      if (!(sj > 0.0) || !isfinite(sj)) ok_s = 0;
      Lm[j * nf + j] = sqrt(fmax(sj, 0.0));
    }
    __syncthreads();
    if (!ok_s) break;
    for (int i = j + 1 + lane; i < nf; i += 64) {
      double t = A[i * nf + j];
      for (int k = 0; k < j; ++k) t -= Lm[i * nf + k] * Lm[j * nf + k];
      Lm[i * nf + j] = t / Lm[j * nf + j];
    }
    __syncthreads();
  }
  if (lane == 0) {
    S.iters += 1;
    if (S.need_jac) {
      S.need_jac = 0;
      S.njev += 1;
    }
    mjac[s] = 0;
    if (!ok_s) {
      S.lambda *= prm.lambda_up;
      S.trial = 0;
      mtrial[s] = 0;
      if (S.lambda > prm.lambda_max) {
        S.active = 0;
        S.status = GF_ENOTCONV;
        S.reason = 4;
      }
    } else {
      for (int i = 0; i < nf; ++i) {
        double t = g[i];
        for (int k = 0; k < i; ++k) t -= Lm[i * nf + k] * y[k];
        y[i] = t / Lm[i * nf + i];
      }
      for (int i = nf - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < nf; ++k) t -= Lm[k * nf + i] * y[k];
        y[i] = t / Lm[i * nf + i];
      }
      for (int p = 0; p < P; ++p) theta_t[d.par + p] = theta[d.par + p];
      for (int a = 0; a < nf; ++a) {
        const int64_t i = d.par + idx[a];
        double v = theta[i] + y[a];
        if (prm.lo && v < prm.lo[i]) v = prm.lo[i];
        if (prm.hi && v > prm.hi[i]) v = prm.hi[i];
        theta_t[i] = v;
      }
      S.trial = 1;
      mtrial[s] = 1;
    }
    st[s] = S;
  }
}

// Accept or reject the trial point, update lambda, test the stop rules and
// count the stamps still active (single workgroup).
__global__ __launch_bounds__(1024) void k_lm_update(const StampDesc *__restrict__ desc, int n, LMParams prm,
                                                    const float2 *__restrict__ chi2t, LMState *__restrict__ st,
                                                    double *__restrict__ theta, const double *__restrict__ theta_t,
                                                    int *__restrict__ mjac, int *__restrict__ mtrial,
                                                    int *__restrict__ active_count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    LMState S = st[s];
    if (!S.active) continue;
    const StampDesc d = desc[s];
    const int P = kNPC * d.ncomp + 1;
    if (S.trial) {
      S.nfev += 1;
      const double c2 = (double)chi2t[s].x + (double)chi2t[s].y;
      S.chi2_trial = c2;
      if (c2 < S.chi2) {
        double step = 0.0;
        for (int p = 0; p < P; ++p) {
          const int64_t i = d.par + p;
          if (prm.free_mask && !prm.free_mask[i]) continue;
          const double sc = fmax(fabs(theta[i]), 1.0);
          step = fmax(step, fabs(theta_t[i] - theta[i]) / sc);
        }
        const double rel = c2 > 0.0 ? (S.chi2 - c2) / c2 : 0.0;
        for (int p = 0; p < P; ++p) theta[d.par + p] = theta_t[d.par + p];
        S.chi2 = c2;
        S.lambda /= prm.lambda_down;
        S.need_jac = 1;
        if (c2 == 0.0) {
          S.active = 0; S.status = GF_OK; S.reason = 3;
        } else if (rel < prm.ftol) {
          S.active = 0; S.status = GF_OK; S.reason = 1;
        } else if (step < prm.xtol) {
          S.active = 0; S.status = GF_OK; S.reason = 2;
        }
      } else {
        S.lambda *= prm.lambda_up;
        if (S.lambda > prm.lambda_max) {
          S.active = 0; S.status = GF_ENOTCONV; S.reason = 4;
        }
      }
    }
    if (S.active && S.iters >= prm.max_iter) {
      S.active = 0; S.status = GF_ENOTCONV; S.reason = 5;
    }
    S.trial = 0;
    mtrial[s] = 0;
    mjac[s] = S.active && S.need_jac;
    st[s] = S;
    mine += S.active;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *active_count = cnt;
}

__global__ void k_lm_result(int n, const LMState *__restrict__ st, gf_lm_result *__restrict__ res) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const LMState S = st[s];
  gf_lm_result r;
  r.chi2 = S.chi2;
  r.lambda = S.lambda;
  r.iters = S.iters;
  r.nfev = S.nfev;
  r.njev = S.njev;
  r.status = S.active ? GF_ENOTCONV : S.status;
  r.reason = S.active ? 5 : S.reason;
  r.pad = 0;
  res[s] = r;
}

hipError_t launch_lm_init(hipStream_t st, const gf_batch *b, double lambda0, const float2 *chi2t, LMState *S,
                          int *mjac, int *mtrial, int *cnt) {
  hipLaunchKernelGGL(k_lm_init, dim3((b->n + 255) / 256), dim3(256), 0, st, b->d_desc, b->n, lambda0, chi2t, S,
                     mjac, mtrial, cnt);
  return hipGetLastError();
}

hipError_t launch_lm_clip(hipStream_t st, int64_t n_par, double *theta, const double *lo, const double *hi,
                          double *theta_t) {
  hipLaunchKernelGGL(k_lm_clip, dim3((unsigned)((n_par + 255) / 256)), dim3(256), 0, st, n_par, theta, lo, hi,
                     theta_t);
  return hipGetLastError();
}

hipError_t launch_lm_solve(hipStream_t st, const gf_batch *b, const float *part, int nacc_stride,
                           const gf_lm_opts *o, LMState *S, double *Ag, const double *theta, double *theta_t,
                           int *mjac, int *mtrial) {
  LMParams prm{o->max_iter, o->lambda_up, o->lambda_down, o->lambda_max, o->ftol, o->xtol, o->lo, o->hi,
               o->free_mask};
  hipLaunchKernelGGL(k_lm_solve, dim3(b->n), dim3(64), 0, st, b->d_desc, b->d_neq_first, part, nacc_stride, prm, S,
                     Ag, theta, theta_t, mjac, mtrial);
  return hipGetLastError();
}

hipError_t launch_lm_update(hipStream_t st, const gf_batch *b, const gf_lm_opts *o, const float2 *chi2t,
                            LMState *S, double *theta, const double *theta_t, int *mjac, int *mtrial, int *cnt) {
  LMParams prm{o->max_iter, o->lambda_up, o->lambda_down, o->lambda_max, o->ftol, o->xtol, o->lo, o->hi,
               o->free_mask};
  hipLaunchKernelGGL(k_lm_update, dim3(1), dim3(1024), 0, st, b->d_desc, b->n, prm, chi2t, S, theta, theta_t, mjac,
                     mtrial, cnt);
  return hipGetLastError();
}

hipError_t launch_lm_result(hipStream_t st, int n, const LMState *S, gf_lm_result *res) {
  hipLaunchKernelGGL(k_lm_result, dim3((n + 255) / 256), dim3(256), 0, st, n, S, res);
  return hipGetLastError();
}

}  // namespace gf

// k_reduce.hip -- step 3 of the fitting loop (comparison of model and
// observation as the sum of squared differences: a transform followed by a
// reduce, Barsdell et al., Sec. 3 item 3) and the reductions behind the
// Levenberg-Marquardt update (steps 4-5), for gfx950.
//
// Sums are FP32 with error-free transformations: each thread keeps a (hi, lo)
// pair updated by TwoSum (Knuth), pairs are combined through wave64 shuffles
// and then across the workgroup's four waves in a fixed order, and a second
// small launch adds the workgroup partials of each stamp in a fixed order.
// Nothing depends on the order in which workgroups run, so results are
// bitwise reproducible.  (No cross-workgroup fences: on this chip a
// device-scope release writes back the L2 of the issuing XCD.)
#include "gf_internal.h"
#include "comp.h"
#include "twosum.h"

namespace gf {

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
// r = sqrt(w) (d - m - sky); per workgroup a (hi, lo) partial of sum r^2.
// A chunk that lies wholly inside a stamp whose image offsets are multiples
// of four floats (pointers 16-byte aligned: vec_ok) moves four pixels per
// 16-byte load, all issued before the first use; the last chunk of a stamp
// takes the scalar path.
constexpr int kChi2Vec = kPixChunk / (4 * kThreads);

template <typename TT>
__global__ __launch_bounds__(kThreads) void k_chi2(const StampDesc *__restrict__ desc, const Work *__restrict__ work,
                                                   const float *__restrict__ model, const TT *__restrict__ theta,
                                                   const float *__restrict__ data, const float *__restrict__ weight,
                                                   float *__restrict__ resid, float2 *__restrict__ part,
                                                   const int32_t *__restrict__ first, const int *__restrict__ mask,
                                                   int vec_ok) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  const float sky = sky_of(theta, d);
  const int npix = d.H * d.W;
  const int p0 = w.unit * kPixChunk;
  F2 acc = {0.f, 0.f};
  if (vec_ok && ((d.pix | d.img) & 3) == 0 && p0 + kPixChunk <= npix) {
    // whole chunk inside the stamp (uniform over the workgroup): every load
    // is unconditional and all of them are in flight before the first use
    const float *mp = model + d.pix, *dp = data + d.img, *wp = weight + d.img;
    float4 mv[kChi2Vec], dv[kChi2Vec], wv[kChi2Vec];
#pragma unroll
    for (int k = 0; k < kChi2Vec; ++k) {
      const int p = p0 + 4 * (k * kThreads + (int)threadIdx.x);
      {   // the model is read once: a streaming (non-temporal) load
        typedef float nf4 __attribute__((ext_vector_type(4)));
        const nf4 t = __builtin_nontemporal_load(reinterpret_cast<const nf4 *>(mp + p));
        mv[k] = make_float4(t.x, t.y, t.z, t.w);
      }
      dv[k] = *reinterpret_cast<const float4 *>(dp + p);
      wv[k] = *reinterpret_cast<const float4 *>(wp + p);
    }
#pragma unroll
    for (int k = 0; k < kChi2Vec; ++k) {
      const int p = p0 + 4 * (k * kThreads + (int)threadIdx.x);
      const float4 r = make_float4(sqrtf(wv[k].x) * (dv[k].x - (mv[k].x + sky)),
                                   sqrtf(wv[k].y) * (dv[k].y - (mv[k].y + sky)),
                                   sqrtf(wv[k].z) * (dv[k].z - (mv[k].z + sky)),
                                   sqrtf(wv[k].w) * (dv[k].w - (mv[k].w + sky)));
      if (resid) *reinterpret_cast<float4 *>(resid + d.pix + p) = r;
      acc = f2_add1(acc, r.x * r.x);
      acc = f2_add1(acc, r.y * r.y);
      acc = f2_add1(acc, r.z * r.z);
      acc = f2_add1(acc, r.w * r.w);
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < kPixChunk / kThreads; ++k) {
      const int p = p0 + k * kThreads + (int)threadIdx.x;
      if (p < npix) {
        const float wt = weight[d.img + p];
        const float r = sqrtf(wt) * (data[d.img + p] - (model[d.pix + p] + sky));
        if (resid) resid[d.pix + p] = r;
        acc = f2_add1(acc, r * r);
      }
    }
  }
  const F2 tot = block_sum(acc);
  if (threadIdx.x == 0) part[first[s] + w.unit] = make_float2(tot.hi, tot.lo);   // the unit's own slot
}

static inline int aligned16(const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// One wave64 per stamp: the workgroup partials of the stamp, added in a fixed
// order (each lane walks its strided share, then a shuffle tree).
__global__ __launch_bounds__(64) void k_pair_final(const int32_t *__restrict__ first, const float2 *__restrict__ part,
                                                   float2 *__restrict__ out, const int *__restrict__ mask) {
  const int s = blockIdx.x;
  if (mask && !mask[s]) return;
  F2 r = {0.f, 0.f};
  for (int u = first[s] + (int)threadIdx.x; u < first[s + 1]; u += 64) {
    const float2 v = part[u];
    F2 t = {v.x, v.y};
    r = f2_add(r, t);
  }
  r = wave_sum(r);
  if (threadIdx.x == 0) out[s] = make_float2(r.hi, r.lo);
}

// chi^2 partials of the direct-path stamps at their slots p->d_c2_first (the
// FFT stamps' partials come from the inverse-row pass).
hipError_t launch_chi2_direct(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *model,
                              const void *theta, bool theta_f64, const float *data, const float *weight,
                              float2 *part, const int *mask, const WorkView *v) {
  const bool view = v && v->rows;   // a view always carries its direct chi^2 list (possibly empty)
  const int n = view ? v->n_pix_direct : (int)p->h_pix_direct.size();
  if (n == 0) return hipSuccess;
  const Work *lst = view ? v->pix_direct : p->d_pix_direct;
  ProfScope ps(st, "k_chi2");
  const int vec_ok = aligned16(model) && aligned16(data) && aligned16(weight);
  if (theta_f64)
    hipLaunchKernelGGL((k_chi2<double>), dim3((unsigned)n), dim3(kThreads), 0, st, b->d_desc, lst, model,
                       (const double *)theta, data, weight, (float *)nullptr, part, p->d_c2_first, mask, vec_ok);
  else
    hipLaunchKernelGGL((k_chi2<float>), dim3((unsigned)n), dim3(kThreads), 0, st, b->d_desc, lst, model,
                       (const float *)theta, data, weight, (float *)nullptr, part, p->d_c2_first, mask, vec_ok);
  return hipGetLastError();
}

// Per-stamp (hi, lo) chi^2 from the partials [first[s], first[s+1]).
hipError_t launch_pair_final(hipStream_t st, int n, const int32_t *first, const float2 *part, float2 *out,
                             const int *mask) {
  ProfScope ps(st, "k_pair_final");
  hipLaunchKernelGGL(k_pair_final, dim3(n), dim3(64), 0, st, first, part, out, mask);
  return hipGetLastError();
}

hipError_t launch_chi2(hipStream_t st, const gf_batch *b, const float *model, const void *theta, bool theta_f64,
                       const float *data, const float *weight, float *resid, float2 *part, unsigned int *counters,
                       float2 *chi2, const int *mask) {
  (void)counters;
  dim3 grid((unsigned)b->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  {
    ProfScope ps(st, "k_chi2");
    const int vec_ok = aligned16(model) && aligned16(data) && aligned16(weight) && aligned16(resid);
    if (theta_f64)
      hipLaunchKernelGGL((k_chi2<double>), grid, blk, 0, st, b->d_desc, b->d_pix, model, (const double *)theta,
                         data, weight, resid, part, b->d_pix_first, mask, vec_ok);
    else
      hipLaunchKernelGGL((k_chi2<float>), grid, blk, 0, st, b->d_desc, b->d_pix, model, (const float *)theta, data,
                         weight, resid, part, b->d_pix_first, mask, vec_ok);
  }
  {
    ProfScope ps(st, "k_pair_final");
    hipLaunchKernelGGL(k_pair_final, dim3(b->n), dim3(64), 0, st, b->d_pix_first, part, chi2, mask);
  }
  return hipGetLastError();
}

// ------------------------------------------------- adjoint helpers
// c = scale * cot * (weight ? sqrt(weight) : 1) on the stamp grid, plus the
// per-chunk sums of c (the sky derivative of the contraction).
__global__ __launch_bounds__(kThreads) void k_cot_prep(const StampDesc *__restrict__ desc,
                                                       const Work *__restrict__ work, const float *__restrict__ cot,
                                                       const float *__restrict__ weight, float scale,
                                                       float *__restrict__ c, const int32_t *__restrict__ first,
                                                       float2 *__restrict__ part) {
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
  if (threadIdx.x == 0) part[first[w.stamp] + w.unit] = make_float2(tot.hi, tot.lo);   // the unit's own slot
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
  hipLaunchKernelGGL(k_cot_prep, grid, blk, 0, st, b->d_desc, b->d_pix, cot, weight, scale, c, b->d_pix_first, spart);
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
// For the stamps flagged in mask, per workgroup chunk of kNeqChunk pixels,
// the Gram matrix of the augmented Jacobian rows x = [j_0 .. j_{P-1}, r, 0..]
// (16 columns: the P parameter derivatives with the sky column equal to 1,
// then the residual r = d - m with m = sky + sum_k Ie_k chan(Ie_k)):
//     G = sum_pixels w x x^T,
// which holds A = J^T W J, g = J^T W r and chi^2 = r^T W r at once.  Each
// wave64 accumulates 16 pixels per step with four v_mfma_f32_16x16x4f32
// (FP32 in, FP32 accumulate): lane (i, k) feeds x_i of pixel k as the A
// operand and w x_i as the B operand.  jc: stamp s, channel ch at
// pix * nchan + ch * H*W (nchan = 7 * the largest component count).
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Orders LDS traffic between the lanes of one wave (LDS operations of a wave
// complete in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// With C2 the workgroup also reduces its chunk's chi^2 of the same model
// (compensated FP32, the residual lanes only) into c2part at the unit's slot.
// T threads per workgroup, one unit each: 256 (four waves of 256 pixels)
// for stamps below kNeqBigPix, 512 (eight waves of 128 pixels) above, where
// a single large stamp has too few units to fill the device with four-wave
// workgroups.  PX parameters follow the sky (the kinematic parameters of a
// cube): column SK = 7 NC is the sky's constant 1, columns above it read
// channel column - 1, column P the residual.
template <int NC, bool C2, int T, int PX = 0>
__global__ __launch_bounds__(T) void k_gram(const StampDesc *__restrict__ desc, const Work *__restrict__ work,
                                            const float *__restrict__ jc, int nchan,
                                            const double *__restrict__ theta, const float *__restrict__ data,
                                            const float *__restrict__ weight, float *__restrict__ part,
                                            const int32_t *__restrict__ first, const int *__restrict__ mask,
                                            float2 *__restrict__ c2part, const float *__restrict__ mie) {
  constexpr int SK = kNPC * NC;
  constexpr int P = SK + 1 + PX;
  constexpr int NW = T / 64;
  static_assert(P + 1 <= 16, "augmented Jacobian must fit 16 columns");
  static_assert(T >= 256 && kNeqChunk % (16 * NW) == 0, "whole 16-pixel groups per wave, 256 reducing threads");
  __shared__ float red[NW][256];
  const Work wk = work[blockIdx.x];
  const int s = wk.stamp;
  if (mask && !mask[s]) return;
  const StampDesc d = desc[s];
  if (d.ncomp != NC) return;
  const int npix = d.H * d.W;
  const float *J = jc + d.pix * (int64_t)nchan;
  float ie[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) ie[k] = (float)theta[d.par + kNPC * k + 2];
  const float sky = (float)theta[d.par + SK];
  // one-component stamps flagged in the mask: the Ie channel and the model
  // from the convolved model mie of this point
  const float *mdl = (NC == 1 && mie && mask && (mask[s] & kMaskModelIe)) ? mie + d.pix : nullptr;
  const float inv_ie = (float)(1.0 / theta[d.par + 2]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  constexpr int per_wave = kNeqChunk / NW;
  const int base = wk.unit * kNeqChunk + wv * per_wave;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  F2 c2acc = {0.f, 0.f};
  // channel read by this lane (clamped for the sky / residual lanes)
  const bool jl = i < SK || (i > SK && i < P);
  const int ich = i < SK ? i : (i > SK && i < P) ? i - 1 : 0;
  // The wave stages 64 pixels at a time in LDS: each lane loads every operand
  // of one pixel (whole rows, coalesced, no value loaded by two lanes), forms
  // its model and residual, and stores the MFMA operands (Jacobian channels,
  // weight, residual, in-stamp flag; zeros past the stamp).  The products
  // then read them four pixels at a time in the same order as lane-loaded
  // operands would give, so the sums are the same.
  constexpr int NJ = P - 1;          // Jacobian channels (every column but the sky's)
  constexpr int NR = NJ + 3;
  // rows padded to 65 floats: a lane's stores of one row hit consecutive
  // banks, and the 16 rows one product reads spread over the banks
  __shared__ float stg[NW][NR][65];
  float (*sg)[65] = stg[wv];
  if (base < npix) {
#pragma unroll 1
    for (int blk = 0; blk < per_wave; blk += 64) {
      const int p = base + blk + lane;
      const bool ok = p < npix;
      const int pc = ok ? p : npix - 1;   // in-bounds address for the straight-line loads
      float jv[NJ];
      float m = sky;
      if (mdl) {
#pragma unroll
        for (int c = 0; c < NJ; ++c)
          if (c != 2) jv[c] = J[(int64_t)c * npix + pc];
        const float mv = mdl[pc];
        jv[2] = mv * inv_ie;
        m = sky + mv;
      } else {
#pragma unroll
        for (int c = 0; c < NJ; ++c) jv[c] = J[(int64_t)c * npix + pc];
#pragma unroll
        for (int c = 0; c < NC; ++c) m = fmaf(ie[c], jv[kNPC * c + 2], m);
      }
      const float wt = weight[d.img + pc], dv = data[d.img + pc];
      wave_sync();   // the previous block's operands have been read
#pragma unroll
      for (int c = 0; c < NJ; ++c) sg[c][lane] = ok ? jv[c] : 0.0f;
      sg[NJ][lane] = ok ? wt : 0.0f;
      sg[NJ + 1][lane] = ok ? dv - m : 0.0f;
      sg[NJ + 2][lane] = ok ? 1.0f : 0.0f;
      wave_sync();
#pragma unroll
      for (int g = 0; g < 64; g += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pg = g + 4 * kk + q;
          const float x = jl ? sg[ich][pg] : (i == SK) ? sg[NJ + 2][pg] : (i == P) ? sg[NJ + 1][pg] : 0.0f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x, sg[NJ][pg] * x, acc, 0, 0, 0);
        }
        if constexpr (C2) {
          // lanes i = 0..3 of each 16-lane group take pixel i of the group
          if (i < 4) {
            const int pg = g + 4 * kk + i;
            const float e = sqrtf(sg[NJ][pg]) * sg[NJ + 1][pg];
            c2acc = f2_add1(c2acc, e * e);
          }
        }
      }
    }
  }
  // lane (col = lane % 16, rows 4*(lane/16) .. +3) holds G[row][col]
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv][(4 * kk + r) * 16 + i] = acc[r];
  __shared__ F2 c2w[NW];
  if constexpr (C2) {
    c2acc = wave_sum(c2acc);
    if (lane == 0) c2w[wv] = c2acc;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const int e = threadIdx.x;  // 256 entries, one per thread
    float v = 0.0f;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) v += red[ww][e];
    part[(int64_t)(first[s] + wk.unit) * 256 + e] = v;   // the unit's own slot
  }
  if constexpr (C2) {
    if (threadIdx.x == 0) {
      F2 t = c2w[0];
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) t = f2_add(t, c2w[ww]);
      c2part[first[s] + wk.unit] = make_float2(t.hi, t.lo);
    }
  }
}

hipError_t launch_normal_eq(hipStream_t st, const gf_batch *b, const float *jc, const double *theta,
                            const float *data, const float *weight, float *part, int nacc_stride, int nchan,
                            const int *mask, const WorkView *v, float2 *c2part, int px, const float *mie) {
  (void)nacc_stride;
  const bool view = v && v->neq;
  const Work *lst = view ? v->neq : b->d_neq;
  const int n = view ? v->n_neq : (int)b->h_neq.size();
  const int nbig = view ? v->n_neq_big : b->n_neq_big;   // the large stamps' units come first
  if (n == 0) return hipSuccess;
  ProfScope ps(st, "k_gram");
  bool has1 = false, has2 = false;
  for (const auto &d : b->h_desc) {
    has1 |= d.ncomp == 1;
    has2 |= d.ncomp == 2;
  }
#define GF_GRAM(NC, C2, T, L, G)                                                                                \
  hipLaunchKernelGGL((k_gram<NC, C2, T>), dim3((unsigned)(G)), dim3(T), 0, st, b->d_desc, L, jc, nchan, theta,   \
                     data, weight, part, b->d_neq_first, mask, c2part, mie)
  if (px == kCubePX) {   // one-component stamps with the cube's kinematic parameters, no chi^2 output
    if (nbig > 0)
      hipLaunchKernelGGL((k_gram<1, false, 512, kCubePX>), dim3((unsigned)nbig), dim3(512), 0, st, b->d_desc, lst,
                         jc, nchan, theta, data, weight, part, b->d_neq_first, mask, (float2 *)nullptr, mie);
    if (n > nbig)
      hipLaunchKernelGGL((k_gram<1, false, 256, kCubePX>), dim3((unsigned)(n - nbig)), dim3(256), 0, st, b->d_desc,
                         lst + nbig, jc, nchan, theta, data, weight, part, b->d_neq_first, mask, (float2 *)nullptr,
                         mie);
    return hipGetLastError();
  }
  if (px != 0) return hipErrorInvalidValue;
#define GF_GRAM_NC(NC)                                                               \
  do {                                                                               \
    if (nbig > 0) {                                                                  \
      if (c2part) GF_GRAM(NC, true, 512, lst, nbig); else GF_GRAM(NC, false, 512, lst, nbig); \
    }                                                                                \
    if (n > nbig) {                                                                  \
      if (c2part) GF_GRAM(NC, true, 256, lst + nbig, n - nbig);                      \
      else GF_GRAM(NC, false, 256, lst + nbig, n - nbig);                            \
    }                                                                                \
  } while (0)
  if (has1) GF_GRAM_NC(1);
  if (has2) GF_GRAM_NC(2);
#undef GF_GRAM_NC
#undef GF_GRAM
  return hipGetLastError();
}


// ------------------------------------------------------------- LM kernels
struct LMParams {
  int32_t max_iter;
  double lambda_up, lambda_down, lambda_max, ftol, xtol;
  const double *lo, *hi;
  const uint8_t *free_mask;
  // component constants kept current for the evaluation kernels (null: not
  // kept): cc_t of the trial point (formed by k_lm_solve), cc_th of the
  // current point (copied from cc_t on acceptance)
  CompC *cc_t, *cc_th;
  const float4 *bn;
  int32_t oversample;
  int32_t model_ie;   // > 0: flag one-component stamps' Jacobian masks with kMaskModelIe, this many channels per parameter
};

// Start: one wave per stamp adds the chi^2 partials of the (clipped) start
// point in the order of k_pair_final (the same value, bit for bit), and its
// first lane sets up the stamp's state.
__global__ __launch_bounds__(64) void k_lm_init(const StampDesc *__restrict__ desc, int n, double lambda0,
                                                const int32_t *__restrict__ first,
                                                const float2 *__restrict__ part, LMState *__restrict__ st,
                                                int *__restrict__ mjac, int *__restrict__ mtrial,
                                                int *__restrict__ active_count, int model_ie) {
  const int s = blockIdx.x;
  if (s == 0 && threadIdx.x == 0) *active_count = n;
  F2 r = {0.f, 0.f};
  for (int u = first[s] + (int)threadIdx.x; u < first[s + 1]; u += 64) {
    const float2 v = part[u];
    F2 t = {v.x, v.y};
    r = f2_add(r, t);
  }
  r = wave_sum(r);
  if (threadIdx.x != 0) return;
  LMState S;
  S.lambda = lambda0;
  S.chi2 = (double)r.hi + (double)r.lo;
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
  mjac[s] = S.active ? (model_ie > 0 && desc[s].ncomp == 1 ? mask_model_ie(model_ie) : 1) : 0;
  mtrial[s] = 0;
}

// One workgroup per active stamp.
//  1. When the Jacobian is new, the workgroup adds the stamp's Gram partials
//     in FP64 (8 slices of 64 threads, each thread owning four entries of
//     the 16 x 16 block; wide loads, because one workgroup reads all of a
//     large stamp's partials; 512 threads, so two workgroups share a CU in
//     batches); A = G[0..P-1][0..P-1] (symmetrised from the
//     lower triangle)
//     and g = G[0..P-1][P] are kept in Ag for the later iterations that reuse
//     this Jacobian.
//  2. The first wave damps the system over the free parameters and factors it
//     (Cholesky; lane i keeps row i in registers, finished rows go through
//     LDS, so only wave-level ordering is needed), then does both triangular
//     solves column by column, broadcasting each finished unknown from its
//     lane.
//  3. It writes the clipped trial point and, when asked, the component
//     constants of the trial point.
// Block 0 also clears the count of active stamps that the update kernel of
// this iteration fills.
// Value of v on lane l (l uniform over the wave).
__device__ __forceinline__ double bcast(double v, int l) {
  const uint64_t b = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l), hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

constexpr int kSolveThreads = 512;
constexpr int kSolveSlices = kSolveThreads / 64;

template <int NC, int PX = 0>
__global__ __launch_bounds__(kSolveThreads) void k_lm_solve(const StampDesc *__restrict__ desc,
                                                       const int32_t *__restrict__ neq_first,
                                                       const float *__restrict__ part, LMParams prm,
                                                       LMState *__restrict__ st, double *__restrict__ Ag,
                                                       const double *__restrict__ theta, double *__restrict__ theta_t,
                                                       int *__restrict__ mjac, int *__restrict__ mtrial,
                                                       int *__restrict__ active_count,
                                                       const Work *__restrict__ list) {
  constexpr int P = kNPC * NC + 1 + PX;
  static_assert(P <= kMaxP, "parameters of a stamp");
  __shared__ double Gp[kSolveSlices][256];
  __shared__ double Gs[256];
  __shared__ double As[P * P];
  __shared__ double Lr[P][P];
  __shared__ double th_s[P], lo_s[P], hi_s[P], g_s[P], dl_s[P], tt_s[P];
  __shared__ int fr_s[P], idx_s[P];
  __shared__ int ok_s;
  __shared__ double inv_s[P];
  const int s = list ? list[blockIdx.x].stamp : (int)blockIdx.x;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) *active_count = 0;
  // independent loads first: descriptor, state and unit range together
  const StampDesc d = desc[s];
  const LMState S0 = st[s];
  const int u0 = neq_first[s], u1 = neq_first[s + 1];
  if (d.ncomp != NC) return;
  LMState S = S0;
  if (!S.active) return;
  double *Ags = Ag + (int64_t)s * (kMaxP * kMaxP + kMaxP);
  if (tid < P) {
    const int64_t i = d.par + tid;
    th_s[tid] = theta[i];
    lo_s[tid] = prm.lo ? prm.lo[i] : -INFINITY;
    hi_s[tid] = prm.hi ? prm.hi[i] : INFINITY;
    fr_s[tid] = prm.free_mask ? (int)prm.free_mask[i] : 1;
    idx_s[tid] = 0;
    dl_s[tid] = 0.0;
  }
  if (S.need_jac) {
    // slice sl (64 threads) adds units u0 + sl, u0 + sl + NS, ... in order,
    // each thread four consecutive entries per 16-byte load, so that a large
    // stamp's partials are read in one round of loads; the slices are then
    // added in a fixed order
    const int e4 = tid & 63, sl = tid >> 6;
    const float *pe = part + 4 * e4;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int ub = u0 + sl; ub < u1; ub += 16 * kSolveSlices) {
      // straight-line loads from clamped addresses; the extra ones weigh 0
      float4 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        v[q] = *reinterpret_cast<const float4 *>(pe + (int64_t)min(ub + q * kSolveSlices, u1 - 1) * 256);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const bool in = ub + q * kSolveSlices < u1;
        a0 += in ? (double)v[q].x : 0.0;
        a1 += in ? (double)v[q].y : 0.0;
        a2 += in ? (double)v[q].z : 0.0;
        a3 += in ? (double)v[q].w : 0.0;
      }
    }
    Gp[sl][4 * e4] = a0;
    Gp[sl][4 * e4 + 1] = a1;
    Gp[sl][4 * e4 + 2] = a2;
    Gp[sl][4 * e4 + 3] = a3;
    __syncthreads();
    if (tid < 256) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kSolveSlices; ++q) t += Gp[q][tid];
      Gs[tid] = t;
    }
  }
  __syncthreads();
  if (tid >= 64) return;   // the rest is the first wave's
  {
    constexpr int NE = (P * P + 63) / 64;
    double v[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = min(tid + q * 64, P * P - 1);
      const int a = e / P, b = e - a * P;
      const int hi = a > b ? a : b, lo = a > b ? b : a;
      v[q] = S.need_jac ? Gs[hi * 16 + lo] : Ags[a * kMaxP + b];
    }
    const double gv = S.need_jac ? Gs[min(tid, P - 1) * 16 + P] : Ags[kMaxP * kMaxP + min(tid, P - 1)];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * 64;
      if (e < P * P) {
        As[e] = v[q];
        if (S.need_jac) Ags[(e / P) * kMaxP + (e % P)] = v[q];
      }
    }
    if (tid < P) {
      g_s[tid] = gv;
      if (S.need_jac) Ags[kMaxP * kMaxP + tid] = gv;
    }
  }
  if (tid == 0) ok_s = 1;
  wave_sync();
  // free parameters in order: lane i < nf works on parameter idx_s[i]
  const bool fr = tid < P && fr_s[tid];
  const uint64_t fm = __ballot(fr);
  const int nf = __popcll(fm);
  if (fr) idx_s[__popcll(fm & ((1ull << tid) - 1ull))] = tid;
  double dmax = fr ? As[tid * P + tid] : 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
  wave_sync();
  const bool mine = tid < nf;
  const int my = mine ? idx_s[tid] : 0;
  double row[P];
#pragma unroll
  for (int k = 0; k < P; ++k) row[k] = (mine && k < nf) ? As[my * P + idx_s[k]] : 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (mine && k == tid) row[k] += S.lambda * fmax(row[k], 1e-12 * dmax);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (j < nf) {
      if (tid == j) {
        double sj = row[j];
#pragma unroll
        for (int k = 0; k < j; ++k) sj -= row[k] * row[k];
        if (!(sj > 0.0) || !isfinite(sj)) ok_s = 0;
        // 1/sqrt(sj) from the hardware estimate and three Newton steps
        // (quadratic convergence: full FP64 precision from any estimate good
        // to 2^-8), shorter on this serial path than a square root and a
        // division
        const double a = fmax(sj, 1e-300);
        double r = __builtin_amdgcn_rsq(a);
#pragma unroll
        for (int nt = 0; nt < 3; ++nt) r = r * fma(-0.5 * a * r, r, 1.5);
        row[j] = a * r;
        inv_s[j] = r;
#pragma unroll
        for (int k = 0; k <= j; ++k) Lr[j][k] = row[k];
      }
      wave_sync();
      if (ok_s && mine && tid > j) {
        double t = row[j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= row[k] * Lr[j][k];
        row[j] = t * inv_s[j];
      }
      wave_sync();
    }
  }
  const bool ok = ok_s != 0;
  if (ok) {
    // L y = g: lane i holds the running right-hand side of row i; y_j is
    // final on lane j once columns 0..j-1 are subtracted.
    double t = mine ? g_s[my] : 0.0;
    double y = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j < nf) {
        const double yj = bcast(t, j) * inv_s[j];
        if (tid == j) y = yj;
        if (mine && tid > j) t -= row[j] * yj;
      }
    }
    // L^T x = y: lane k needs column k of L, L[i][k] for i >= k.
    double col[P];
#pragma unroll
    for (int i = 0; i < P; ++i) col[i] = (mine && i < nf && tid <= i) ? Lr[i][tid] : 0.0;
    double u = y, x = 0.0;
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {
      if (i < nf) {
        const double xi = bcast(u, i) * inv_s[i];
        if (tid == i) x = xi;
        if (mine && tid < i) u -= col[i] * xi;
      }
    }
    if (mine) dl_s[my] = x;
  }
  if (tid == 0) {
    S.iters += 1;
    if (S.need_jac) {
      S.need_jac = 0;
      S.njev += 1;
    }
    mjac[s] = 0;
    if (!ok) {
      S.lambda *= prm.lambda_up;
      S.trial = 0;
      mtrial[s] = 0;
      if (S.lambda > prm.lambda_max) {
        S.active = 0;
        S.status = GF_ENOTCONV;
        S.reason = 4;
      }
    } else {
      S.trial = 1;
      mtrial[s] = 1;
    }
    st[s] = S;
  }
  wave_sync();
  // trial point theta' = clip(theta + delta) on the free parameters
  if (ok && tid < P) {
    double v = th_s[tid];
    if (fr) v = fmin(fmax(v + dl_s[tid], lo_s[tid]), hi_s[tid]);
    theta_t[d.par + tid] = v;
    tt_s[tid] = v;
  }
  if (PX == 0 && prm.cc_t) {
    wave_sync();
    if (ok && tid < NC)
      comp_setup<double>(tt_s + kNPC * tid, prm.bn, prm.oversample, prm.cc_t[(int64_t)s * kMaxComp + tid]);
  }
}

// Finish the trial chi^2 of every active stamp (one wave per stamp: its
// workgroup partials added in a fixed order), accept or reject the trial
// point, update lambda, test the stop rules, and count the stamps still
// active.
__global__ __launch_bounds__(64) void k_lm_update(const StampDesc *__restrict__ desc,
                                                  const int32_t *__restrict__ pix_first,
                                                  const float2 *__restrict__ part, LMParams prm,
                                                  LMState *__restrict__ st, double *__restrict__ theta,
                                                  const double *__restrict__ theta_t, int *__restrict__ mjac,
                                                  int *__restrict__ mtrial, int *__restrict__ active_count,
                                                  const Work *__restrict__ list) {
  const int s = list ? list[blockIdx.x].stamp : (int)blockIdx.x;
  LMState S = st[s];
  if (!S.active) return;
  const StampDesc d = desc[s];
  const int P = d.P;
  const int lane = threadIdx.x;
  double c2 = 0.0;
  double stp = 0.0;
  double th = 0.0, tt = 0.0;
  if (S.trial) {
    F2 r = {0.f, 0.f};
    for (int u = pix_first[s] + lane; u < pix_first[s + 1]; u += 64) {
      const float2 v = part[u];
      F2 t = {v.x, v.y};
      r = f2_add(r, t);
    }
    r = wave_sum(r);
    c2 = (double)r.hi + (double)r.lo;
    if (lane < P) {
      const int64_t i = d.par + lane;
      th = theta[i];
      tt = theta_t[i];
      if (!prm.free_mask || prm.free_mask[i]) stp = fabs(tt - th) / fmax(fabs(th), 1.0);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) stp = fmax(stp, __shfl_xor(stp, off, 64));
  }
  const bool accept = S.trial && c2 < S.chi2;
  if (accept && lane < P) theta[d.par + lane] = tt;
  if (accept && prm.cc_t) {
    const int nw = d.ncomp * (int)(sizeof(CompC) / sizeof(uint32_t));
    const uint32_t *src = reinterpret_cast<const uint32_t *>(prm.cc_t + (int64_t)s * kMaxComp);
    uint32_t *dst = reinterpret_cast<uint32_t *>(prm.cc_th + (int64_t)s * kMaxComp);
    for (int q = lane; q < nw; q += 64) dst[q] = src[q];
  }
  if (lane != 0) return;
  if (S.trial) {
    S.nfev += 1;
    S.chi2_trial = c2;
    if (accept) {
      const double rel = c2 > 0.0 ? (S.chi2 - c2) / c2 : 0.0;
      S.chi2 = c2;
      S.lambda /= prm.lambda_down;
      S.need_jac = 1;
      if (c2 == 0.0) {
        S.active = 0; S.status = GF_OK; S.reason = 3;
      } else if (rel < prm.ftol) {
        S.active = 0; S.status = GF_OK; S.reason = 1;
      } else if (stp < prm.xtol) {
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
  mjac[s] = (S.active && S.need_jac) ? (prm.model_ie > 0 && d.ncomp == 1 ? mask_model_ie(prm.model_ie) : 1) : 0;
  st[s] = S;
  if (S.active) atomicAdd(active_count, 1);
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

// Per observation group: the member with the lowest chi^2 among converged
// members (among all members if none converged); ties go to the lower stamp
// index, NaN never wins.  One thread per group.
__global__ void k_group_best(const StampDesc *__restrict__ desc, int G, const int32_t *__restrict__ gfirst,
                             const int32_t *__restrict__ gmembers, const gf_lm_result *__restrict__ res,
                             const double *__restrict__ theta, double *__restrict__ best, int32_t *__restrict__ best_stamp) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int pick = -1;
  for (int pass = 0; pass < 2 && pick < 0; ++pass) {
    double bc = INFINITY;
    for (int i = gfirst[g]; i < gfirst[g + 1]; ++i) {
      const int s = gmembers[i];
      if (pass == 0 && res[s].status != GF_OK) continue;
      const double c = res[s].chi2;
      if (!(c < bc)) continue;   // NaN and ties lose: the lowest index wins
      bc = c;
      pick = s;
    }
  }
  if (pick < 0) pick = gmembers[gfirst[g]];   // every chi^2 infinite or NaN
  if (best_stamp) best_stamp[g] = pick;
  double *o = best + (int64_t)g * kMaxP;
  const int P = kNPC * desc[pick].ncomp + 1;
  for (int q = 0; q < kMaxP; ++q) o[q] = q < P ? theta[desc[pick].par + q] : 0.0;
}

hipError_t launch_group_best(hipStream_t st, const gf_batch *b, const gf_lm_result *res, const double *theta,
                             double *best, int32_t *best_stamp) {
  ProfScope ps(st, "k_group_best");
  hipLaunchKernelGGL(k_group_best, dim3((b->n_groups + 255) / 256), dim3(256), 0, st, b->d_desc, b->n_groups,
                     b->d_gfirst, b->d_gmembers, res, theta, best, best_stamp);
  return hipGetLastError();
}

// Starting points of a multi-start fit of single-Sersic stamps: start k of
// group g is theta0[g] with rule k applied: 0 unchanged, 1 n = 1 and Re x 1.5,
// 2 n = 4 and Re x 0.7, 3 phi + pi/2 (mod pi).
__global__ void k_expand_starts(int G, int S, const double *__restrict__ theta0, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G * S) return;
  const int g = i / S, k = i - g * S;
  double t[8];
  for (int q = 0; q < 8; ++q) t[q] = theta0[8 * (int64_t)g + q];
  if (k == 1) {
    t[4] = 1.0;
    t[3] *= 1.5;
  } else if (k == 2) {
    t[4] = 4.0;
    t[3] *= 0.7;
  } else if (k == 3) {
    t[6] = fmod(t[6] + 1.5707963267948966, 3.141592653589793);
    if (t[6] < 0.0) t[6] += 3.141592653589793;
  }
  for (int q = 0; q < 8; ++q) out[8 * (int64_t)i + q] = t[q];
}

hipError_t launch_expand_starts(hipStream_t st, int G, int S, const double *theta0, double *out) {
  if (G * S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_starts, dim3((G * S + 255) / 256), dim3(256), 0, st, G, S, theta0, out);
  return hipGetLastError();
}

// Restricted work lists: workgroup r copies piece r of the plan.
__global__ __launch_bounds__(64) void k_copy_runs(const CopyRun *__restrict__ plan, Work *__restrict__ dst) {
  const CopyRun r = plan[blockIdx.x];
  for (int i = (int)threadIdx.x; i < r.len; i += 64) dst[r.dst_off + i] = r.src[i];
}

hipError_t launch_copy_runs(hipStream_t st, const CopyRun *plan, int n, Work *dst) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_runs, dim3((unsigned)n), dim3(64), 0, st, plan, dst);
  return hipGetLastError();
}

hipError_t launch_lm_init(hipStream_t st, const gf_batch *b, double lambda0, const int32_t *first,
                          const float2 *part, LMState *S, int *mjac, int *mtrial, int *cnt, int model_ie) {
  hipLaunchKernelGGL(k_lm_init, dim3((unsigned)b->n), dim3(64), 0, st, b->d_desc, b->n, lambda0, first, part, S, mjac,
                     mtrial, cnt, model_ie);
  return hipGetLastError();
}

hipError_t launch_lm_solve(hipStream_t st, const gf_batch *b, const float *part, const gf_lm_opts *o, LMState *S,
                           double *Ag, const double *theta, double *theta_t, int *mjac, int *mtrial, int *cnt,
                           CompC *cc_th, CompC *cc_t, const float4 *bn, const WorkView *v, int px) {
  LMParams prm{o->max_iter, o->lambda_up, o->lambda_down, o->lambda_max, o->ftol, o->xtol, o->lo, o->hi,
               o->free_mask, cc_t, cc_th, bn, o->oversample, 0};
  ProfScope ps(st, "k_lm_solve");
  bool has1 = false, has2 = false;
  for (const auto &d : b->h_desc) {
    has1 |= d.ncomp == 1;
    has2 |= d.ncomp == 2;
  }
  // a compacted view lists the stamps still iterating; the others would
  // only start and end a workgroup
  const Work *list = v && v->stamps ? v->stamps : nullptr;
  const unsigned grid = list ? (unsigned)v->n_stamps : (unsigned)b->n;
  if (grid == 0) return hipSuccess;
  if (px == kCubePX) {
    hipLaunchKernelGGL((k_lm_solve<1, kCubePX>), dim3(grid), dim3(kSolveThreads), 0, st, b->d_desc, b->d_neq_first,
                       part, prm, S, Ag, theta, theta_t, mjac, mtrial, cnt, list);
    return hipGetLastError();
  }
  if (px != 0) return hipErrorInvalidValue;
  if (has1)
    hipLaunchKernelGGL((k_lm_solve<1>), dim3(grid), dim3(kSolveThreads), 0, st, b->d_desc, b->d_neq_first, part,
                       prm, S, Ag, theta, theta_t, mjac, mtrial, cnt, list);
  if (has2)
    hipLaunchKernelGGL((k_lm_solve<2>), dim3(grid), dim3(kSolveThreads), 0, st, b->d_desc, b->d_neq_first, part,
                       prm, S, Ag, theta, theta_t, mjac, mtrial, cnt, list);
  return hipGetLastError();
}

hipError_t launch_lm_update(hipStream_t st, const gf_batch *b, const gf_lm_opts *o, const int32_t *first,
                            const float2 *part, LMState *S, double *theta, const double *theta_t, int *mjac,
                            int *mtrial, int *cnt, CompC *cc_th, CompC *cc_t, const WorkView *v, int model_ie) {
  LMParams prm{o->max_iter, o->lambda_up, o->lambda_down, o->lambda_max, o->ftol, o->xtol, o->lo, o->hi,
               o->free_mask, cc_t, cc_th, nullptr, o->oversample, model_ie};
  ProfScope ps(st, "k_lm_update");
  const Work *list = v && v->stamps ? v->stamps : nullptr;
  const unsigned grid = list ? (unsigned)v->n_stamps : (unsigned)b->n;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lm_update, dim3(grid), dim3(64), 0, st, b->d_desc, first, part, prm, S, theta,
                     theta_t, mjac, mtrial, cnt, list);
  return hipGetLastError();
}

hipError_t launch_lm_result(hipStream_t st, int n, const LMState *S, gf_lm_result *res) {
  hipLaunchKernelGGL(k_lm_result, dim3((n + 255) / 256), dim3(256), 0, st, n, S, res);
  return hipGetLastError();
}

}  // namespace gf

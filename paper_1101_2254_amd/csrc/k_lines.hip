// k_lines.hip -- spectral-line fitting: steps 1-3 and the Levenberg-Marquardt
// loop in one dimension (Barsdell et al., Sec. 5: spectral-line fitting is
// the same transform / convolve / reduce problem once the dimensionality may
// change), for gfx950.
//
// One workgroup of 256 threads owns one spectrum.  Output channels are
// processed in chunks of 256: the sub-sampled Gaussian lines (and, for the
// Jacobian, their three derivatives per line) are evaluated on the chunk's
// padded channels into LDS, then each thread convolves its own output
// channel with the line-spread function held in LDS.  Spectra are short
// (hundreds to a few thousand channels), so the direct sum over at most
// GF_LINE_MAX_K taps is the convolution of choice and nothing leaves the
// workgroup.  The fit kernel keeps the whole LM state of its spectrum on chip
// and iterates until the spectrum stops: one launch fits the whole batch,
// with no host round trips and no idle workgroups for finished spectra.
#include "gf_internal.h"
#include "twosum.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace gf {

constexpr int kLT = 256;                         // threads; output channels per chunk
constexpr int kLinePadW = kLT + GF_LINE_MAX_K - 1;

// Per-line constants.  The centre is split into the nearest integer channel
// and a fraction, and the sub-sample offsets relative to the fraction,
//   (s + 1/2)/S - 1/2 - f = ((2s + 1 - S) - 2S f) / (2S),
// take one FMA and one division, so x - mu keeps full relative precision
// near the line centre whatever the channel index.
struct LineC {
  int32_t mi;
  float fo[GF_MAX_OVERSAMPLE];
  float a;      // peak
  float k2;     // -log2(e) / (2 sigma^2)
  float isg2;   // 1 / sigma^2
  float isg3;   // 1 / sigma^3
};

template <typename TT>
__device__ void line_setup(const TT *t3, int S, LineC &c) {
  const TT mu = t3[1];
  const TT mr = rint(mu);
  c.mi = (int)mr;
  const float f = (float)(mu - mr);
  const float twoS = 2.0f * (float)S;
  for (int a = 0; a < S; ++a) c.fo[a] = fmaf(-twoS, f, (float)(2 * a + 1 - S)) / twoS;
  const float sg = (float)t3[2];
  c.a = (float)t3[0];
  c.k2 = -1.4426950408889634f / (2.0f * sg * sg);
  c.isg2 = 1.0f / (sg * sg);
  c.isg3 = c.isg2 / sg;
}

// Fills channel planes of the padded chunk: plane 0 the model (sub-sample
// mean of the sum of the lines), planes 1 + 3k .. 3 + 3k the derivatives in
// (A, mu, sigma) of line k when JAC.  Padded channel j of the spectrum sits at
// x = j - c; the chunk starting at output channel i0 covers padded channels
// i0 .. i0 + n_out + K - 2.
template <int L, bool JAC>
__device__ void line_chunk_eval(const LineC *__restrict__ lc, int S, int K, int i0, int n_out,
                                float (*__restrict__ pv)[kLinePadW]) {
  const int c = (K - 1) >> 1;
  const float invS = 1.0f / (float)S;
  const int np = n_out + K - 1;
  for (int t = (int)threadIdx.x; t < np; t += kLT) {
    const int xc = i0 + t - c;
    float m = 0.0f;
    float ga[L], gm[L], gs[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const float base = (float)(xc - lc[k].mi);
      const float a = lc[k].a, k2 = lc[k].k2;
      float fo[GF_MAX_OVERSAMPLE];
#pragma unroll
      for (int s = 0; s < GF_MAX_OVERSAMPLE; ++s) fo[s] = lc[k].fo[s];
      float sg = 0.0f, sm = 0.0f, ss = 0.0f;
#pragma unroll
      for (int s = 0; s < GF_MAX_OVERSAMPLE; ++s) {
        if (s < S) {
          const float dx = base + fo[s];
          const float g = __builtin_amdgcn_exp2f(dx * dx * k2);
          sg += g;
          if (JAC) {
            const float gd = g * dx;
            sm += gd;
            ss = fmaf(gd, dx, ss);
          }
        }
      }
      m = fmaf(a, sg, m);
      ga[k] = sg * invS;
      gm[k] = a * sm * invS * lc[k].isg2;
      gs[k] = a * ss * invS * lc[k].isg3;
    }
    pv[0][t] = m * invS;
    if (JAC) {
#pragma unroll
      for (int k = 0; k < L; ++k) {
        pv[1 + 3 * k][t] = ga[k];
        pv[2 + 3 * k][t] = gm[k];
        pv[3 + 3 * k][t] = gs[k];
      }
    }
  }
}

// Valid convolution of planes 0 .. NP-1 at this thread's output channel
// (tid < n_out): every plane shares each tap load, and the loop is unrolled
// so that the LDS loads of several taps are in flight together.
template <int NP>
__device__ __forceinline__ void line_conv(const float *__restrict__ lsf, int K, const float (*__restrict__ pv)[kLinePadW],
                                          int tid, float *v) {
#pragma unroll
  for (int q = 0; q < NP; ++q) v[q] = 0.0f;
  const int b = tid + K - 1;
#pragma unroll 4
  for (int u = 0; u < K; ++u) {
    const float l = lsf[u];
#pragma unroll
    for (int q = 0; q < NP; ++q) v[q] = fmaf(l, pv[q][b - u], v[q]);
  }
}

// Fixed-order compensated workgroup sum (waves in order).
__device__ F2 line_block_sum(F2 v, F2 *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  F2 r = red[0];
#pragma unroll
  for (int q = 1; q < kLT / 64; ++q) r = f2_add(r, red[q]);
  return r;
}

// chi^2 of the spectrum at the constants lc (model = conv + continuum).
template <int L>
__device__ F2 line_chi2_pass(const LineC *lc, float cont, int S, int N, int K, const float *lsf_s,
                             const float *__restrict__ dp, const float *__restrict__ wp,
                             float (*pv)[kLinePadW], F2 *red) {
  F2 acc = {0.f, 0.f};
  for (int i0 = 0; i0 < N; i0 += kLT) {
    const int n_out = min(kLT, N - i0);
    line_chunk_eval<L, false>(lc, S, K, i0, n_out, pv);
    __syncthreads();
    const int tid = threadIdx.x;
    if (tid < n_out) {
      float mc;
      line_conv<1>(lsf_s, K, pv, tid, &mc);
      const float m = mc + cont;
      const float r = sqrtf(wp[i0 + tid]) * (dp[i0 + tid] - m);
      acc = f2_add1(acc, r * r);
    }
    __syncthreads();
  }
  return line_block_sum(acc, red);
}

// ------------------------------------------------------- model and chi^2
template <int L, typename TT>
__global__ __launch_bounds__(kLT) void k_line_model(const LineDesc *__restrict__ desc, int n,
                                                    const float *__restrict__ lsf, const TT *__restrict__ theta,
                                                    int S, float *__restrict__ out) {
  __shared__ float lsf_s[GF_LINE_MAX_K];
  __shared__ float pv[1][kLinePadW];
  __shared__ LineC lc[L];
  const int sp = blockIdx.x;
  if (sp >= n) return;
  const LineDesc d = desc[sp];
  if (d.nl != L) return;
  const int tid = threadIdx.x;
  if (tid < d.K) lsf_s[tid] = lsf[d.lsf + tid];
  if (tid < L) line_setup<TT>(theta + d.par + 3 * tid, S, lc[tid]);
  __syncthreads();
  const float cont = (float)theta[d.par + 3 * L];
  for (int i0 = 0; i0 < d.N; i0 += kLT) {
    const int n_out = min(kLT, d.N - i0);
    line_chunk_eval<L, false>(lc, S, d.K, i0, n_out, pv);
    __syncthreads();
    if (tid < n_out) {
      float mc;
      line_conv<1>(lsf_s, d.K, pv, tid, &mc);
      out[d.data + i0 + tid] = mc + cont;
    }
    __syncthreads();
  }
}

template <int L, typename TT>
__global__ __launch_bounds__(kLT) void k_line_chi2(const LineDesc *__restrict__ desc, int n,
                                                   const float *__restrict__ lsf, const TT *__restrict__ theta,
                                                   int S, const float *__restrict__ data,
                                                   const float *__restrict__ weight, float2 *__restrict__ out) {
  __shared__ float lsf_s[GF_LINE_MAX_K];
  __shared__ float pv[1][kLinePadW];
  __shared__ LineC lc[L];
  __shared__ F2 red[kLT / 64];
  const int sp = blockIdx.x;
  if (sp >= n) return;
  const LineDesc d = desc[sp];
  if (d.nl != L) return;
  const int tid = threadIdx.x;
  if (tid < d.K) lsf_s[tid] = lsf[d.lsf + tid];
  if (tid < L) line_setup<TT>(theta + d.par + 3 * tid, S, lc[tid]);
  __syncthreads();
  const F2 c2 = line_chi2_pass<L>(lc, (float)theta[d.par + 3 * L], S, d.N, d.K, lsf_s, data + d.data,
                                  weight + d.data, pv, red);
  if (tid == 0) out[sp] = make_float2(c2.hi, c2.lo);
}

// ------------------------------------------------------------------- fit
// Every iteration of the rule of the image fits, per spectrum:
//   A = J^T W J, g = J^T W (d - m) over the free parameters (the Gram matrix
//   of [J 1 r] weighted by w, FP32 per thread, FP64 across the workgroup),
//   (A + lambda diag(max(A_ii, 1e-12 max A_jj))) delta = g by FP64 Cholesky
//   (not positive definite: lambda *= up), theta' = clip(theta + delta),
//   accept iff chi2(theta') < chi2(theta) (compensated FP32 sums).
// Registers capped for as many waves per SIMD as the LDS of each build allows
// workgroups per CU: six for one line, five for two, four for three
// (uncapped the three-line build took 139 VGPRs, three waves).
template <int L>
__global__ __launch_bounds__(kLT) __attribute__((amdgpu_waves_per_eu(L == 1 ? 6 : L == 2 ? 5 : 4)))
void k_line_lm(const LineDesc *__restrict__ desc, int n, const float *__restrict__ lsf, const float *__restrict__ data,
               const float *__restrict__ weight, double *__restrict__ theta, LineLMParams prm,
               gf_lm_result *__restrict__ res) {
  constexpr int P = 3 * L + 1;    // parameters; the continuum is the last
  static_assert(P + 1 <= 16, "the Gram block holds 16 columns");
  __shared__ float lsf_s[GF_LINE_MAX_K];
  __shared__ float pv[3 * L + 1][kLinePadW];
  __shared__ LineC lc[L];
  __shared__ F2 red[kLT / 64];
  __shared__ float xs[kLT][17];            // sqrt(w) [J 1 r] of a chunk (row stride 17: no bank conflicts)
  // per-wave Gram blocks, in the chunk staging buffer (free once a Jacobian's
  // chunks are done), so the LDS of a workgroup stays smaller
  float(*gw)[256] = reinterpret_cast<float(*)[256]>(&xs[0][0]);
  __shared__ double Gs[256];                // Gram matrix G[a][b] at a * 16 + b
  __shared__ double th_s[P], tt_s[P], lo_s[P], hi_s[P], dl_s[P];
  __shared__ double Lr[P][P], inv_s[P];
  __shared__ int fr_s[P], idx_s[P];
  __shared__ int ok_s, go_s;
  const int sp = blockIdx.x;
  if (sp >= n) return;
  const LineDesc d = desc[sp];
  if (d.nl != L) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float *dp = data + d.data, *wp = weight + d.data;
  if (tid < d.K) lsf_s[tid] = lsf[d.lsf + tid];
  if (tid < P) {
    const int64_t i = d.par + tid;
    const double lo = prm.lo ? prm.lo[i] : -INFINITY, hi = prm.hi ? prm.hi[i] : INFINITY;
    lo_s[tid] = lo;
    hi_s[tid] = hi;
    fr_s[tid] = prm.free_mask ? (int)prm.free_mask[i] : 1;
    th_s[tid] = fmin(fmax(theta[i], lo), hi);   // the start is clipped too
  }
  __syncthreads();
  if (tid < L) line_setup<double>(th_s + 3 * tid, prm.S, lc[tid]);
  __syncthreads();
  F2 c2p = line_chi2_pass<L>(lc, (float)th_s[P - 1], prm.S, d.N, d.K, lsf_s, dp, wp, pv, red);
  double chi2 = (double)c2p.hi + (double)c2p.lo;
  double lambda = prm.lambda0;
  int iters = 0, nfev = 1, njev = 0, status = GF_ENOTCONV, reason = 5;
  bool need_jac = true;
  if (chi2 == 0.0) {
    status = GF_OK;
    reason = 3;
  }
  // free parameters in order: lane i < nf of wave 0 works on idx_s[i]
  if (tid < P) idx_s[tid] = 0;
  __syncthreads();
  const bool frl = tid < P && fr_s[tid];
  const uint64_t fm = __ballot(frl);   // wave 0 holds every parameter lane
  const int nf = __popcll(fm);
  if (wv == 0 && frl) idx_s[__popcll(fm & ((1ull << tid) - 1ull))] = tid;
  __syncthreads();
  for (int it = 1; reason == 5 && status != GF_OK && it <= prm.max_iter; ++it) {
    iters = it;
    if (need_jac) {
      // ---- Gram matrix of [J r] at theta (lc holds theta's constants)
      // Per chunk every thread stages sqrt(w) [J 1 r] of its channel in LDS
      // and each wave adds the 16 x 16 Gram block of its 64 channels with
      // v_mfma_f32_16x16x4f32 (lane (i, k) feeds column i of channel k as
      // both operands); the accumulator stays in four registers per lane.
      floatx4 gacc = {0.f, 0.f, 0.f, 0.f};
      const float cont = (float)th_s[P - 1];
      const int gi = lane & 15, gk = lane >> 4;
      for (int i0 = 0; i0 < d.N; i0 += kLT) {
        const int n_out = min(kLT, d.N - i0);
        line_chunk_eval<L, true>(lc, prm.S, d.K, i0, n_out, pv);
        __syncthreads();
        float y[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) y[q] = 0.0f;
        if (tid < n_out) {
          float cv[3 * L + 1];
          line_conv<3 * L + 1>(lsf_s, d.K, pv, tid, cv);
          const float sw = sqrtf(wp[i0 + tid]);
#pragma unroll
          for (int q = 0; q < 3 * L; ++q) y[q] = sw * cv[1 + q];
          y[P - 1] = sw;
          y[P] = sw * (dp[i0 + tid] - (cv[0] + cont));
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) xs[tid][q] = y[q];
        __syncthreads();
#pragma unroll
        for (int g = 0; g < 64; g += 16) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float v = xs[64 * wv + g + 4 * gk + q][gi];
            gacc = __builtin_amdgcn_mfma_f32_16x16x4f32(v, v, gacc, 0, 0, 0);
          }
        }
        __syncthreads();
      }
      // lane (col = lane % 16, rows 4 (lane / 16) .. +3) holds G[row][col]
#pragma unroll
      for (int r = 0; r < 4; ++r) gw[wv][(4 * gk + r) * 16 + gi] = gacc[r];
      __syncthreads();
      {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kLT / 64; ++q) t += (double)gw[q][tid];
        Gs[tid] = t;
      }
      __syncthreads();
      ++njev;
      need_jac = false;
    }
    // ---- damped Cholesky and solve (first wave; lane i holds row i)
    if (wv == 0) {
      const bool mine = lane < nf;
      const int my = mine ? idx_s[lane] : 0;
      auto Gat = [&](int a, int b) -> double { return Gs[a * 16 + b]; };
      double dmax = (lane < P && fr_s[lane]) ? Gat(lane, lane) : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
      double row[P];
#pragma unroll
      for (int k = 0; k < P; ++k) row[k] = (mine && k < nf) ? Gat(my, idx_s[k]) : 0.0;
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (mine && k == lane) row[k] += lambda * fmax(row[k], 1e-12 * dmax);
      if (lane == 0) ok_s = 1;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < P; ++j) {
        if (j < nf) {
          if (lane == j) {
            double sj = row[j];
#pragma unroll
            for (int k = 0; k < j; ++k) sj -= row[k] * row[k];
            if (!(sj > 0.0) || !isfinite(sj)) ok_s = 0;
            const double dj = sqrt(fmax(sj, 0.0));
            row[j] = dj;
            inv_s[j] = 1.0 / dj;
#pragma unroll
            for (int k = 0; k <= j; ++k) Lr[j][k] = row[k];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (ok_s && mine && lane > j) {
            double t = row[j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= row[k] * Lr[j][k];
            row[j] = t * inv_s[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      if (ok_s) {
        double t = mine ? Gat(my, P) : 0.0;   // g = J^T W r
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (j < nf) {
            const double yj = __shfl(t, j, 64) * inv_s[j];
            if (lane == j) y = yj;
            if (mine && lane > j) t -= row[j] * yj;
          }
        }
        double col[P];
#pragma unroll
        for (int i = 0; i < P; ++i) col[i] = (mine && i < nf && lane <= i) ? Lr[i][lane] : 0.0;
        double u = y, xs = 0.0;
#pragma unroll
        for (int i = P - 1; i >= 0; --i) {
          if (i < nf) {
            const double xi = __shfl(u, i, 64) * inv_s[i];
            if (lane == i) xs = xi;
            if (mine && lane < i) u -= col[i] * xi;
          }
        }
        if (lane < P) dl_s[lane] = 0.0;
        __builtin_amdgcn_wave_barrier();
        if (mine) dl_s[my] = xs;
      }
    }
    __syncthreads();
    if (!ok_s) {
      lambda *= prm.lambda_up;
      if (lambda > prm.lambda_max) {
        status = GF_ENOTCONV;
        reason = 4;
      }
      // every wave has read the flag before the first wave's next solve
      // sets it again
      __syncthreads();
      continue;
    }
    // ---- trial point and its chi^2
    if (tid < P) {
      double v = th_s[tid];
      if (fr_s[tid]) v = fmin(fmax(v + dl_s[tid], lo_s[tid]), hi_s[tid]);
      tt_s[tid] = v;
    }
    __syncthreads();
    if (tid < L) line_setup<double>(tt_s + 3 * tid, prm.S, lc[tid]);
    __syncthreads();
    const F2 ct = line_chi2_pass<L>(lc, (float)tt_s[P - 1], prm.S, d.N, d.K, lsf_s, dp, wp, pv, red);
    const double c2t = (double)ct.hi + (double)ct.lo;
    ++nfev;
    if (c2t < chi2) {
      double step = 0.0;
      for (int p = 0; p < P; ++p)
        if (fr_s[p]) step = fmax(step, fabs(tt_s[p] - th_s[p]) / fmax(fabs(th_s[p]), 1.0));
      const double rel = c2t > 0.0 ? (chi2 - c2t) / c2t : 0.0;
      __syncthreads();
      if (tid < P) th_s[tid] = tt_s[tid];   // lc already holds the accepted point's constants
      chi2 = c2t;
      lambda /= prm.lambda_down;
      need_jac = true;
      if (chi2 == 0.0) {
        status = GF_OK;
        reason = 3;
      } else if (rel < prm.ftol) {
        status = GF_OK;
        reason = 1;
      } else if (step < prm.xtol) {
        status = GF_OK;
        reason = 2;
      }
    } else {
      lambda *= prm.lambda_up;
      if (lambda > prm.lambda_max) {
        status = GF_ENOTCONV;
        reason = 4;
      }
      __syncthreads();
      if (tid < L) line_setup<double>(th_s + 3 * tid, prm.S, lc[tid]);   // back to theta's constants
    }
    __syncthreads();
  }
  if (tid < P) theta[d.par + tid] = th_s[tid];
  if (tid == 0) {
    gf_lm_result r;
    r.chi2 = chi2;
    r.lambda = lambda;
    r.iters = iters;
    r.nfev = nfev;
    r.njev = njev;
    r.status = status;
    r.reason = reason;
    r.pad = 0;
    res[sp] = r;
  }
}

// ------------------------------------------------------------- launchers
hipError_t launch_line_model(hipStream_t st, const gf_line_batch *lb, const float *lsf, const float *theta, int S,
                             float *out) {
  ProfScope ps(st, "k_line_model");
  for (int L = 1; L <= GF_LINE_MAX_LINES; ++L) {
    if (!lb->has_nl[L]) continue;
    if (L == 1)
      hipLaunchKernelGGL((k_line_model<1, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S, out);
    else if (L == 2)
      hipLaunchKernelGGL((k_line_model<2, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S, out);
    else
      hipLaunchKernelGGL((k_line_model<3, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S, out);
  }
  return hipGetLastError();
}

hipError_t launch_line_chi2(hipStream_t st, const gf_line_batch *lb, const float *lsf, const float *theta, int S,
                            const float *data, const float *weight, float2 *out) {
  ProfScope ps(st, "k_line_chi2");
  for (int L = 1; L <= GF_LINE_MAX_LINES; ++L) {
    if (!lb->has_nl[L]) continue;
    if (L == 1)
      hipLaunchKernelGGL((k_line_chi2<1, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S,
                         data, weight, out);
    else if (L == 2)
      hipLaunchKernelGGL((k_line_chi2<2, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S,
                         data, weight, out);
    else
      hipLaunchKernelGGL((k_line_chi2<3, float>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, theta, S,
                         data, weight, out);
  }
  return hipGetLastError();
}

// One kernel per line count present, each on its own stream (the kernels
// differ in register use, so running them side by side keeps every CU busy
// through each kernel's tail of slow spectra).
hipError_t launch_line_lm(const hipStream_t *sts, const gf_line_batch *lb, const float *lsf, const float *data,
                          const float *weight, double *theta, const LineLMParams &prm, gf_lm_result *res) {
  for (int L = 1; L <= GF_LINE_MAX_LINES; ++L) {
    if (!lb->has_nl[L]) continue;
    hipStream_t st = sts[L - 1];
    if (L == 1)
      hipLaunchKernelGGL((k_line_lm<1>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, data, weight, theta,
                         prm, res);
    else if (L == 2)
      hipLaunchKernelGGL((k_line_lm<2>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, data, weight, theta,
                         prm, res);
    else
      hipLaunchKernelGGL((k_line_lm<3>), dim3(lb->n), dim3(kLT), 0, st, lb->d_desc, lb->n, lsf, data, weight, theta,
                         prm, res);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gf

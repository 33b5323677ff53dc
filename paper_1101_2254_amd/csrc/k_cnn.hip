// k_cnn.hip -- kernels of the learned starting-point proposal: a small
// convolutional network that maps a 128 x 128 stamp to the eight parameters
// of a single Sersic component plus sky, trained on rendered stamps.
//
// Layout: activations NHWC in BF16; each 3x3 stride-2 padding-1 convolution
// is an im2col gather followed by a GEMM on the matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation); weights are kept as FP32
// master copies with BF16 mirrors in the same flat layout.  Backward passes
// reuse the same GEMM with transposed operand addressing and split-K partial
// sums reduced in a fixed order, so every result is bit-reproducible.
#include "gf_internal.h"

namespace gf {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (inputs are finite)
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Eight BF16 values moved as one 16-byte word.
union alignas(16) B8 {
  uint4 u;
  bf16_t h[8];
};

// ------------------------------------------------------------------ GEMM
// C(m, n) = sum_k A(m, k) B(n, k) with
//   A(m, k) = A[m*lda + k] if AK else A[k*lda + m]
//   B(n, k) = B[n*ldb + k] if BK else B[k*ldb + n]
// Tiles of 64 x BN x 32 per workgroup of four waves; split-K over gridDim.z.
constexpr int kGemmBM = 64, kGemmBK = 32, kGemmLdsK = kGemmBK + 8;

__device__ __forceinline__ void epi_store(const Epi &e, int m, int n, float v) {
  if (e.bias) v += e.bias[n];
  if (e.relu) v = fmaxf(v, 0.f);
  if (e.mask && !(bf2f(e.mask[(int64_t)m * e.ldm + n]) > 0.f)) v = 0.f;
  if (e.outf) e.outf[(int64_t)m * e.ldf + n] = v;
  if (e.outb) e.outb[(int64_t)m * e.ldb + n] = f2bf(v);
}

// Stage rows [r0, r0+ROWS) x k [k0, k0+32) of an operand into S[row][k].
template <bool KC, int ROWS>
__device__ __forceinline__ void gemm_stage(const bf16_t *__restrict__ g, int ld, int r0, int k0, int R, int kend,
                                           bf16_t (*S)[kGemmLdsK]) {
  if (KC) {
    for (int e = threadIdx.x * 8; e < ROWS * kGemmBK; e += 256 * 8) {
      const int r = e / kGemmBK, kc = e - r * kGemmBK;
      const int gr = r0 + r, gk = k0 + kc;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gr < R) {
        const bf16_t *p = g + (int64_t)gr * ld + gk;
        if (gk + 8 <= kend) {
          v = *reinterpret_cast<const uint4 *>(p);
        } else {
          B8 t;
          for (int j = 0; j < 8; ++j) t.h[j] = gk + j < kend ? p[j] : (bf16_t)0;
          v = t.u;
        }
      }
      *reinterpret_cast<uint4 *>(&S[r][kc]) = v;
    }
  } else {
    for (int e = threadIdx.x * 8; e < ROWS * kGemmBK; e += 256 * 8) {
      const int kk = e / ROWS, rc = e - kk * ROWS;
      const int gk = k0 + kk, gr = r0 + rc;
      B8 t;
      t.u = make_uint4(0, 0, 0, 0);
      if (gk < kend) {
        const bf16_t *p = g + (int64_t)gk * ld + gr;
        if (gr + 8 <= R) {
          t.u = *reinterpret_cast<const uint4 *>(p);
        } else {
          for (int j = 0; j < 8; ++j) t.h[j] = gr + j < R ? p[j] : (bf16_t)0;
        }
      }
      for (int j = 0; j < 8; ++j) S[rc + j][kk] = t.h[j];
    }
  }
}

template <bool AK, bool BK, int BN>
__global__ __launch_bounds__(256) void k_gemm(const bf16_t *__restrict__ A, int lda, const bf16_t *__restrict__ B,
                                              int ldb, int M, int N, int K, int kchunk, Epi epi,
                                              float *__restrict__ part) {
  constexpr int WM = BN == 64 ? 2 : 4, WN = 4 / WM;
  constexpr int TM = kGemmBM / WM / 16, TN = BN / WN / 16;
  __shared__ __attribute__((aligned(16))) bf16_t As[kGemmBM][kGemmLdsK];
  __shared__ __attribute__((aligned(16))) bf16_t Bs[BN][kGemmLdsK];
  const int m0 = blockIdx.x * kGemmBM, n0 = blockIdx.y * BN;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WN) * (kGemmBM / WM), wn0 = (wave % WN) * (BN / WN);
  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int li = lane & 15, lk = 4 * (lane >> 4);
  for (int k0 = kb; k0 < ke; k0 += kGemmBK) {
    gemm_stage<AK, kGemmBM>(A, lda, m0, k0, M, ke, As);
    gemm_stage<BK, BN>(B, ldb, n0, k0, N, ke, Bs);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 16) {
      v4s af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const v4s *>(&As[wm0 + i * 16 + li][kk + lk]);
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *reinterpret_cast<const v4s *>(&Bs[wn0 + j * 16 + li][kk + lk]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element r of tile (i, j): row 4*(lane/16) + r, column lane % 16
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + i * 16 + lk + r, n = n0 + wn0 + j * 16 + li;
        if (m >= M || n >= N) continue;
        if (part)
          part[((int64_t)blockIdx.z * M + m) * N + n] = acc[i][j][r];
        else
          epi_store(epi, m, n, acc[i][j][r]);
      }
}

// Sum of `n` values at stride `stride` in index order, with the loads of
// eight values in flight at a time (the additions keep the same order).
__device__ __forceinline__ float ordered_sum(const float *__restrict__ p, int n, int64_t stride) {
  float s = 0.f;
  int z = 0;
  for (; z + 8 <= n; z += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(z + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; z < n; ++z) s += p[(int64_t)z * stride];
  return s;
}

// Sum of split-K partials in split order, then the epilogue.
__global__ void k_gemm_reduce(const float *__restrict__ part, int splits, int M, int N, Epi epi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const float s = ordered_sum(part + i, splits, (int64_t)M * N);
  epi_store(epi, (int)(i / N), (int)(i % N), s);
}

// ------------------------------------------------------------------ layout kernels
// Per-stamp mean and 1/standard deviation (population) of the outer frame of
// `border` pixels; an all-constant frame gives 1/sd = 1.
__global__ __launch_bounds__(256) void k_border_stats(const float *__restrict__ x, int side, int border,
                                                      float2 *__restrict__ stats) {
  __shared__ double red[256];
  const float *p = x + (int64_t)blockIdx.x * side * side;
  const int inner = side - 2 * border;
  double s = 0.0;
  for (int i = threadIdx.x; i < side * side; i += 256) {
    const int r = i / side, c = i - r * side;
    if (r >= border && r < side - border && c >= border && c < side - border) continue;
    s += p[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double cnt = (double)side * side - (double)inner * inner;
  const double mean = red[0] / cnt;
  __syncthreads();
  double q = 0.0;
  for (int i = threadIdx.x; i < side * side; i += 256) {
    const int r = i / side, c = i - r * side;
    if (r >= border && r < side - border && c >= border && c < side - border) continue;
    const double d = p[i] - mean;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sd = sqrt(red[0] / cnt);
    stats[blockIdx.x] = make_float2((float)mean, sd > 0.0 ? (float)(1.0 / sd) : 1.f);
  }
}

// First-layer columns: row (n, oy, ox) holds the nine taps
// asinh((x - mean) / sd) at (2oy+ky-1, 2ox+kx-1) (zero outside), then seven zeros.
__global__ void k_im2col_first(const float *__restrict__ x, const float2 *__restrict__ stats, int nb, int side,
                               bf16_t *__restrict__ col) {
  const int ho = side / 2;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int64_t)nb * ho * ho) return;
  const int s = (int)(row / (ho * ho));
  const int rem = (int)(row - (int64_t)s * ho * ho);
  const int oy = rem / ho, ox = rem - oy * ho;
  const float2 st = stats[s];
  const float *p = x + (int64_t)s * side * side;
  B8 v[2];
  v[0].u = make_uint4(0, 0, 0, 0);
  v[1].u = make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int ky = 0; ky < 3; ++ky)
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1, tap = ky * 3 + kx;
      if (iy >= 0 && iy < side && ix >= 0 && ix < side)
        v[tap >> 3].h[tap & 7] = f2bf(asinhf((p[iy * side + ix] - st.x) * st.y));
    }
  uint4 *o = reinterpret_cast<uint4 *>(col + row * 16);
  o[0] = v[0].u;
  o[1] = v[1].u;
}

// Columns of a 3x3 stride-2 padding-1 convolution over NHWC x [nb][H][H][C]
// (C % 8 == 0): row (n, oy, ox), column (ky*3 + kx)*C + c.
__global__ void k_im2col(const bf16_t *__restrict__ x, int nb, int H, int C, bf16_t *__restrict__ col) {
  const int ho = H / 2, cv = C / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nb * ho * ho * 9 * cv;
  if (i >= total) return;
  const int c8 = (int)(i % cv);
  const int64_t t = i / cv;
  const int tap = (int)(t % 9);
  const int64_t row = t / 9;
  const int s = (int)(row / (ho * ho));
  const int rem = (int)(row - (int64_t)s * ho * ho);
  const int oy = rem / ho, ox = rem - oy * ho;
  const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (iy >= 0 && iy < H && ix >= 0 && ix < H)
    v = *reinterpret_cast<const uint4 *>(x + (((int64_t)s * H + iy) * H + ix) * C + c8 * 8);
  *reinterpret_cast<uint4 *>(col + row * 9 * C + tap * C + c8 * 8) = v;
}

// Adjoint of k_im2col fused with the ReLU derivative: for input pixel
// (n, iy, ix, c), sum the column entries that read it, keep the sum where the
// layer's activation act > 0, write BF16.
__global__ void k_col2im_relu(const float *__restrict__ dcol, const bf16_t *__restrict__ act, int nb, int H, int C,
                              bf16_t *__restrict__ dx) {
  const int ho = H / 2, cv = C / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nb * H * H * cv;
  if (i >= total) return;
  const int c8 = (int)(i % cv);
  const int64_t pix = i / cv;
  const int s = (int)(pix / (H * H));
  const int rem = (int)(pix - (int64_t)s * H * H);
  const int iy = rem / H, ix = rem - iy * H;
  float acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.f;
  // iy = 2 oy + ky - 1: even iy -> ky = 1; odd iy -> (ky = 0, oy = (iy+1)/2) and (ky = 2, oy = (iy-1)/2)
  int oys[2], kys[2], ny = 0, oxs[2], kxs[2], nx = 0;
  if ((iy & 1) == 0) { oys[0] = iy / 2; kys[0] = 1; ny = 1; }
  else {
    if ((iy + 1) / 2 < ho) { oys[ny] = (iy + 1) / 2; kys[ny] = 0; ++ny; }
    oys[ny] = (iy - 1) / 2; kys[ny] = 2; ++ny;
  }
  if ((ix & 1) == 0) { oxs[0] = ix / 2; kxs[0] = 1; nx = 1; }
  else {
    if ((ix + 1) / 2 < ho) { oxs[nx] = (ix + 1) / 2; kxs[nx] = 0; ++nx; }
    oxs[nx] = (ix - 1) / 2; kxs[nx] = 2; ++nx;
  }
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      const int64_t row = ((int64_t)s * ho + oys[a]) * ho + oxs[b];
      const float *p = dcol + row * 9 * C + (kys[a] * 3 + kxs[b]) * C + c8 * 8;
      const float4 u = *reinterpret_cast<const float4 *>(p), w = *reinterpret_cast<const float4 *>(p + 4);
      acc[0] += u.x; acc[1] += u.y; acc[2] += u.z; acc[3] += u.w;
      acc[4] += w.x; acc[5] += w.y; acc[6] += w.z; acc[7] += w.w;
    }
  const int64_t o = pix * C + c8 * 8;
  B8 av, r;
  av.u = *reinterpret_cast<const uint4 *>(act + o);
#pragma unroll
  for (int j = 0; j < 8; ++j) r.h[j] = bf2f(av.h[j]) > 0.f ? f2bf(acc[j]) : (bf16_t)0;
  *reinterpret_cast<uint4 *>(dx + o) = r.u;
}

// Column sums of an M x N matrix (N divides 256), rows split into chunks of
// `rows_per` rows: partial[chunk][n].
template <typename T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<bf16_t>(bf16_t v) { return bf2f(v); }

template <typename T>
__global__ __launch_bounds__(256) void k_colsum_part(const T *__restrict__ x, int M, int N, int rows_per,
                                                     float *__restrict__ part) {
  __shared__ float red[256];
  const int g = 256 / N, c = threadIdx.x % N, rg = threadIdx.x / N;
  const int r0 = blockIdx.x * rows_per, r1 = min(M, r0 + rows_per);
  float s = 0.f;
  for (int r = r0 + rg; r < r1; r += g) s += to_f<T>(x[(int64_t)r * N + c]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (rg == 0) {
    float t = 0.f;
    for (int q = 0; q < g; ++q) t += red[q * N + c];
    part[(int64_t)blockIdx.x * N + c] = t;
  }
}

// BF16 matrices with N % 8 == 0: each thread adds 16-byte vectors of eight
// columns over a strided subset of the chunk's rows; the row groups are then
// added in a fixed order.
__global__ __launch_bounds__(256) void k_colsum_part_v8(const bf16_t *__restrict__ x, int M, int N, int rows_per,
                                                        float *__restrict__ part) {
  __shared__ float red[256 * 8];
  const int cv = N / 8, g = 256 / cv, c8 = threadIdx.x % cv, rg = threadIdx.x / cv;
  const int r0 = blockIdx.x * rows_per, r1 = min(M, r0 + rows_per);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int r = r0 + rg; r < r1; r += g) {
    B8 v;
    v.u = *reinterpret_cast<const uint4 *>(x + (int64_t)r * N + c8 * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] += bf2f(v.h[j]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[rg * N + c8 * 8 + j] = acc[j];
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += 256) {
    float t = 0.f;
    for (int q = 0; q < g; ++q) t += red[q * N + c];
    part[(int64_t)blockIdx.x * N + c] = t;
  }
}

__global__ void k_colsum_final(const float *__restrict__ part, int chunks, int N, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  out[c] = ordered_sum(part + c, chunks, N);
}

// Mean squared error over nb x 8 outputs; dy = 2 (y - t) / (8 nb).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, int n,
                                             float *__restrict__ dy, bf16_t *__restrict__ dyb,
                                             float *__restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float d = y[i] - t[i];
    s += (double)d * d;
    const float g = sc * d;
    dy[i] = g;
    dyb[i] = f2bf(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = (float)(red[0] / n);
}

// Adam with bias-corrected moments; c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, bf16_t *__restrict__ pb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ p, bf16_t *__restrict__ pb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

// ------------------------------------------------------------------ parameter coding
// Regression targets of a single Sersic component plus sky on a side-N stamp:
//   t0 = x0 - N/2, t1 = y0 - N/2,
//   t2 = (ln Ie - m_I)/h_I over [0.5, 5], t3 = (ln Re - m_R)/h_R over [2, N/4],
//   t4 = (n - 3.25)/2.75, (t5, t6) = (1 - q)(cos 2 phi, sin 2 phi)/0.8,
//   t7 = (sky - 0.025)/0.025.
struct Box {
  double mi, hi, mr, hr;
};
__device__ __forceinline__ Box box_for(int side) {
  const double l05 = log(0.5), l5 = log(5.0), l2 = log(2.0), lr = log(0.25 * side);
  return Box{0.5 * (l05 + l5), 0.5 * (l5 - l05), 0.5 * (l2 + lr), 0.5 * (lr - l2)};
}

__global__ void k_encode(int n, int side, const float *__restrict__ theta, float *__restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Box b = box_for(side);
  const float *p = theta + 8 * (int64_t)i;
  float *o = t + 8 * (int64_t)i;
  const double e = 1.0 - p[5];
  double s2, c2;
  sincos(2.0 * (double)p[6], &s2, &c2);
  o[0] = (float)(p[0] - 0.5 * side);
  o[1] = (float)(p[1] - 0.5 * side);
  o[2] = (float)((log((double)p[2]) - b.mi) / b.hi);
  o[3] = (float)((log((double)p[3]) - b.mr) / b.hr);
  o[4] = (float)((p[4] - 3.25) / 2.75);
  o[5] = (float)(e * c2 / 0.8);
  o[6] = (float)(e * s2 / 0.8);
  o[7] = (float)((p[7] - 0.025) / 0.025);
}

// Inverse of k_encode into FP64 starting points: n clamped to [0.2, 10],
// ellipticity 1 - q clamped to [0, 0.95], phi wrapped to [0, pi).
__global__ void k_decode(int n, int side, const float *__restrict__ t, double *__restrict__ theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Box b = box_for(side);
  const float *p = t + 8 * (int64_t)i;
  double *o = theta + 8 * (int64_t)i;
  o[0] = 0.5 * side + p[0];
  o[1] = 0.5 * side + p[1];
  o[2] = exp(b.mi + b.hi * p[2]);
  o[3] = exp(b.mr + b.hr * p[3]);
  o[4] = fmin(10.0, fmax(0.2, 3.25 + 2.75 * p[4]));
  const double e1 = 0.8 * p[5], e2 = 0.8 * p[6];
  o[5] = 1.0 - fmin(0.95, sqrt(e1 * e1 + e2 * e2));
  double phi = 0.5 * atan2(e2, e1);
  if (phi < 0.0) phi += 3.141592653589793;
  o[6] = phi;
  o[7] = 0.025 + 0.025 * p[7];
}

// ------------------------------------------------------------------ launchers
static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_gemm(hipStream_t st, bool ak, bool bk, const bf16_t *A, int lda, const bf16_t *B, int ldb, int M,
                       int N, int K, const Epi &epi, float *part, int64_t part_cap) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int bn = N <= 32 ? 32 : 64;
  const int tm = (M + kGemmBM - 1) / kGemmBM, tn = (N + bn - 1) / bn;
  int splits = 1;
  const int kb = (K + kGemmBK - 1) / kGemmBK;
  if (tm * tn < 512 && part) {
    splits = std::min((512 + tm * tn - 1) / (tm * tn), std::max(1, kb / 8));   // >= 8 k-steps per split
    while (splits > 1 && (int64_t)splits * M * N > part_cap) --splits;
  }
  const int kchunk = ((kb + splits - 1) / splits) * kGemmBK;
  splits = (K + kchunk - 1) / kchunk;
  if (splits < 1) splits = 1;
  float *pp = splits > 1 ? part : nullptr;
  dim3 grid(tm, tn, splits);
  ProfScope ps(st, "k_gemm_bf16");
#define GF_GEMM(AKV, BKV, BNV) \
  hipLaunchKernelGGL((k_gemm<AKV, BKV, BNV>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, kchunk, epi, pp)
  if (ak && bk) { if (bn == 32) GF_GEMM(true, true, 32); else GF_GEMM(true, true, 64); }
  else if (ak && !bk) { if (bn == 32) GF_GEMM(true, false, 32); else GF_GEMM(true, false, 64); }
  else if (!ak && !bk) { if (bn == 32) GF_GEMM(false, false, 32); else GF_GEMM(false, false, 64); }
  else { if (bn == 32) GF_GEMM(false, true, 32); else GF_GEMM(false, true, 64); }
#undef GF_GEMM
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  hipLaunchKernelGGL(k_gemm_reduce, dim3(nblk((int64_t)M * N)), dim3(256), 0, st, part, splits, M, N, epi);
  return hipGetLastError();
}

hipError_t launch_border_stats(hipStream_t st, const float *x, int nb, int side, int border, float2 *stats) {
  ProfScope ps(st, "k_border_stats");
  hipLaunchKernelGGL(k_border_stats, dim3(nb), dim3(256), 0, st, x, side, border, stats);
  return hipGetLastError();
}

hipError_t launch_im2col_first(hipStream_t st, const float *x, const float2 *stats, int nb, int side, bf16_t *col) {
  const int64_t rows = (int64_t)nb * (side / 2) * (side / 2);
  ProfScope ps(st, "k_im2col_first");
  hipLaunchKernelGGL(k_im2col_first, dim3(nblk(rows)), dim3(256), 0, st, x, stats, nb, side, col);
  return hipGetLastError();
}

hipError_t launch_im2col(hipStream_t st, const bf16_t *x, int nb, int H, int C, bf16_t *col) {
  const int64_t n = (int64_t)nb * (H / 2) * (H / 2) * 9 * (C / 8);
  ProfScope ps(st, "k_im2col");
  hipLaunchKernelGGL(k_im2col, dim3(nblk(n)), dim3(256), 0, st, x, nb, H, C, col);
  return hipGetLastError();
}

hipError_t launch_col2im_relu(hipStream_t st, const float *dcol, const bf16_t *act, int nb, int H, int C,
                              bf16_t *dx) {
  const int64_t n = (int64_t)nb * H * H * (C / 8);
  ProfScope ps(st, "k_col2im_relu");
  hipLaunchKernelGGL(k_col2im_relu, dim3(nblk(n)), dim3(256), 0, st, dcol, act, nb, H, C, dx);
  return hipGetLastError();
}

hipError_t launch_colsum(hipStream_t st, const void *x, bool is_bf16, int M, int N, float *part, float *out) {
  const int rows_per = 2048;
  const int chunks = (M + rows_per - 1) / rows_per;
  ProfScope ps(st, "k_colsum");
  if (is_bf16 && N % 8 == 0 && 256 % (N / 8) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0)
    hipLaunchKernelGGL(k_colsum_part_v8, dim3(chunks), dim3(256), 0, st, (const bf16_t *)x, M, N, rows_per, part);
  else if (is_bf16)
    hipLaunchKernelGGL(k_colsum_part<bf16_t>, dim3(chunks), dim3(256), 0, st, (const bf16_t *)x, M, N, rows_per, part);
  else
    hipLaunchKernelGGL(k_colsum_part<float>, dim3(chunks), dim3(256), 0, st, (const float *)x, M, N, rows_per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3(nblk(N)), dim3(256), 0, st, part, chunks, N, out);
  return hipGetLastError();
}

int colsum_chunks(int M) { return (M + 2047) / 2048; }

hipError_t launch_mse(hipStream_t st, const float *y, const float *t, int n, float *dy, bf16_t *dyb, float *loss) {
  ProfScope ps(st, "k_mse");
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, y, t, n, dy, dyb, loss);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, int64_t n, float *p, const float *g, float *m, float *v, bf16_t *pb, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  ProfScope ps(st, "k_adam");
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, st, n, p, g, m, v, pb, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(hipStream_t st, int64_t n, const float *p, bf16_t *pb) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, st, n, p, pb);
  return hipGetLastError();
}

hipError_t launch_encode(hipStream_t st, int n, int side, const float *theta, float *t) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode, dim3(nblk(n)), dim3(256), 0, st, n, side, theta, t);
  return hipGetLastError();
}

hipError_t launch_decode(hipStream_t st, int n, int side, const float *t, double *theta) {
  if (n <= 0) return hipSuccess;
  ProfScope ps(st, "k_decode");
  hipLaunchKernelGGL(k_decode, dim3(nblk(n)), dim3(256), 0, st, n, side, t, theta);
  return hipGetLastError();
}

}  // namespace gf

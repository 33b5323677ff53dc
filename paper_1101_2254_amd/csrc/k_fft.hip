// k_fft.hip -- step 2 of the fitting loop in Fourier space (Barsdell et al.,
// Sec. 3 item 2: FFT plus a pointwise transform), hand-written for gfx950.
//
// The linear convolution of an Mh x Mw padded grid with a K x K PSF is taken
// from the circular convolution on an L x L grid with L >= max(Mh, Mw): the
// kept "valid" rows and columns K-1 .. M-1 never see a wrapped tap.  Three
// launches per convolution, each a batch of independent 1-D transforms held in
// one LDS buffer of fft_cap(RMAX) complex values per workgroup:
//   rows   : two real rows per complex transform (z = a + i b), length L,
//            split into the half spectra A, B (L/2+1 bins) -> spectra S1[row][k]
//   columns: per bin k, forward transform over rows, times the OTF (or its
//            conjugate for the adjoint correlation), inverse transform, keep
//            the wanted rows -> S2[row][k]
//   irows  : rebuild two Hermitian spectra as Z = A + i B, inverse transform,
//            real part -> first row, imaginary part -> second row, crop.
// The 1/L^2 of the inverse transform is folded into the OTF.
//
// Transforms are mixed-radix Stockham passes done in place in LDS, with FP32
// pass twiddles that the host computes in FP64.  A pass's radix is computed
// in registers: 2, 3, 4, 5 and 8 directly, and the composites 6 ... 32 by one
// Cooley-Tukey split with compile-time twiddles, so the transform sizes of
// the workloads (48 ... 576) take two LDS passes each.
#include <utility>

#include "gf_internal.h"
#include "bufload.h"
#include "fft_dft.h"
#include "twosum.h"

namespace gf {

__device__ __forceinline__ int fdiv(int x, uint32_t m) { return m ? (int)__umulhi((uint32_t)x, m) : x; }

// Division of x < 2^16 by a divisor fixed for the whole workgroup.
struct FDiv {
  uint32_t m;
  __device__ __forceinline__ explicit FDiv(int d) : m(d <= 1 ? 0u : 0xffffffffu / (uint32_t)d + 1u) {}
  __device__ __forceinline__ int operator()(int x) const { return fdiv(x, m); }
};

// LDS index with one padding slot per 32 complex values: the strided
// accesses of the early Stockham passes (stride R) then spread over the banks.
__device__ __forceinline__ int lp(int i) { return i + (i >> 5); }
constexpr int fft_lds(int cap) { return cap + cap / 32 + 1; }
// Loops that move up to the buffer's capacity between memory and LDS are unrolled
// this many times so each thread issues all of its global loads before it
// waits on any of them.  The loads go through range-checked buffer
// resources: an element outside the valid region gets an out-of-range
// offset and reads zero, so no load sits under a branch (a load under a
// branch makes the compiler wait for it inside the branch, which turns the
// batch into one round trip per load).
constexpr int fft_iters(int cap) { return (cap + kThreads - 1) / kThreads; }
constexpr int kTwIters = (GF_MAX_FFT + kThreads - 1) / kThreads;

// Stage the L twiddles of a plan into LDS (loads first, then stores).
__device__ __forceinline__ void stage_twiddles(float2 *tw, const float2 *__restrict__ src, int L) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, (uint32_t)L * 8u);
  float2 t[kTwIters];
#pragma unroll
  for (int it = 0; it < kTwIters; ++it) {
    const int i = (int)threadIdx.x + it * kThreads;
    t[it] = bload_f32x2(rs, (uint32_t)i * 8u);
  }
#pragma unroll
  for (int it = 0; it < kTwIters; ++it) {
    const int i = (int)threadIdx.x + it * kThreads;
    if (i < L) tw[i] = t[it];
  }
}

// One in-place Stockham pass over T transforms of length L (stride Ls).
// Butterfly j of a transform reads x[j + r L/R], twiddles input r by
// W_{Ns R}^{r k} (k = j mod Ns), does a radix-R DFT in registers and writes to
// (j div Ns) Ns R + k + r Ns.  Every thread first loads all of its
// butterflies (NB of them: T L <= CAP guarantees one round), the
// workgroup synchronises, and then all results are stored, so a single LDS
// buffer suffices.  For R > 8 the twiddle of input r is formed as
// W^{(r mod 8) k} W^{8 (r div 8) k} from two table entries.
template <int R, bool INV, int CAP>
__device__ __forceinline__ void stockham_pass(float2 *__restrict__ buf, int T, int L, int Ls, int Ns, uint32_t ns_m,
                                              uint32_t nb_m, const float2 *__restrict__ tw) {
  constexpr int NB = (CAP + kThreads * R - 1) / (kThreads * R);
  const int nb = L / R;
  const int total = T * nb;
  const int twstep = L / (Ns * R);
  float2 v[NB][R];
  int dst[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int idx = (int)threadIdx.x + b * (int)blockDim.x;
    dst[b] = -1;
    if (idx < total) {
      const int t = fdiv(idx, nb_m);
      const int j = idx - t * nb;
      const int jd = fdiv(j, ns_m);
      const int k = j - jd * Ns;
      const int src = t * Ls + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[lp(src + r * nb)];
      if (Ns > 1) {
        const int ks = k * twstep;
        if constexpr (R <= 8) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const float2 w = tw[r * ks];
            v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
          }
        } else {
          float2 lo[8], hi[(R + 7) / 8];
          lo[0] = make_float2(1.f, 0.f);
#pragma unroll
          for (int a = 1; a < 8; ++a) lo[a] = tw[a * ks];
          hi[0] = make_float2(1.f, 0.f);
#pragma unroll
          for (int c = 1; c < (R + 7) / 8; ++c) hi[c] = tw[8 * c * ks];
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const float2 w = (r >= 8) ? ((r & 7) ? cmul(lo[r & 7], hi[r >> 3]) : hi[r >> 3]) : lo[r];
            v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
          }
        }
      }
      dft<R, INV>(v[b]);
      dst[b] = t * Ls + jd * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (dst[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(dst[b] + r * Ns)] = v[b][r];
    }
  }
  __syncthreads();
}

// Full transform of T transforms in place (T * L <= fft_cap(RMAX)).  RMAX is the
// largest radix the kernel is built for (18, 24 or 32): plans of small radices
// run in kernels without the larger register butterflies, which need fewer
// registers and so keep more waves per SIMD.
template <bool INV, int RMAX>
__device__ __forceinline__ void lds_fft(float2 *buf, int T, int Ls, const FftPlan &pl, const float2 *tw) {
  constexpr int CAP = fft_cap(RMAX);
  const int L = pl.L;
  for (int s = 0; s < pl.nstages; ++s) {
    const int R = pl.radix[s], Ns = pl.ns[s];
    const uint32_t nsm = pl.ns_magic[s], nbm = pl.nb_magic[s];
    switch (R) {
      case 2: stockham_pass<2, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 3: stockham_pass<3, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 4: stockham_pass<4, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 5: stockham_pass<5, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 6: stockham_pass<6, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 8: stockham_pass<8, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 9: stockham_pass<9, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 10: stockham_pass<10, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 12: stockham_pass<12, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 15: stockham_pass<15, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 16: stockham_pass<16, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      case 18: stockham_pass<18, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
      default:
        if constexpr (RMAX > 18) {
          switch (R) {
            case 20: stockham_pass<20, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
            case 24: stockham_pass<24, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
            default:
              if constexpr (RMAX > 24) {
                switch (R) {
                  case 25: stockham_pass<25, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
                  case 27: stockham_pass<27, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
                  default: stockham_pass<32, INV, CAP>(buf, T, L, Ls, Ns, nsm, nbm, tw); break;
                }
              }
              break;
          }
        }
        break;
    }
  }
}

// Geometry of one launch mode (the modes are listed in gf_internal.h).

struct Geo {
  int in_rows, in_cols, in_col0;   // row pass input (cols placed at in_col0 on the L grid)
  int col_row0;                    // rows of S1 placed at this row of the L grid
  int out_row0, out_rows;          // column pass keeps rows out_row0 .. +out_rows (all L for OTF)
  int out_col0, out_cols;          // inverse row pass keeps these columns
};

__device__ __forceinline__ Geo geo_of(int mode, const StampDesc &d, int L) {
  Geo g;
  const int km1 = d.K - 1;
  if (mode == MODE_CONV || mode == MODE_CHI2) {
    g.in_rows = d.Mh; g.in_cols = d.Mw; g.in_col0 = 0; g.col_row0 = 0;
    g.out_row0 = km1; g.out_rows = d.H; g.out_col0 = km1; g.out_cols = d.W;
  } else if (mode == MODE_CORR) {
    g.in_rows = d.H; g.in_cols = d.W; g.in_col0 = km1; g.col_row0 = km1;
    g.out_row0 = 0; g.out_rows = d.Mh; g.out_col0 = 0; g.out_cols = d.Mw;
  } else {
    g.in_rows = d.K; g.in_cols = d.K; g.in_col0 = 0; g.col_row0 = 0;
    g.out_row0 = 0; g.out_rows = L; g.out_col0 = 0; g.out_cols = 0;
  }
  return g;
}

// Spectra are stored bin-major ("transposed"): S1 of a channel is
// [L/2+1 bins][in_rows rows] and S2 is [L/2+1 bins][out_rows rows], so the
// column pass reads and writes whole contiguous columns and the row passes
// exchange runs of 2T consecutive rows per bin.  Row transforms sit in LDS with
// stride L+1 (odd in units of 8 bytes), so the bin-major exchanges hit
// distinct LDS banks.

// ------------------------------------------------------------ row pass
// in: real images; stamp s channel ch starts at in_base(s) * n_ch + ch * plane.
// S1: stamp s channel ch starts at s1_off[s] * n_ch + ch * (L/2+1) * in_rows.
template <int MODE, int RMAX>
__global__ __launch_bounds__(kThreads) void k_fft_rows(const StampDesc *__restrict__ desc,
                                                       const PathDesc *__restrict__ path,
                                                       const FftPlan *__restrict__ plans,
                                                       const float2 *__restrict__ tw_all,
                                                       const Work *__restrict__ work, const float *__restrict__ in,
                                                       int n_ch, const int64_t *__restrict__ s1_off,
                                                       float2 *__restrict__ S1, const int *__restrict__ mask,
                                                       int tmax) {
  extern __shared__ float2 lds[];
  constexpr int CAP = fft_cap(RMAX), LDS0 = fft_lds(CAP), NIT = fft_iters(CAP);
  const Work w = work[blockIdx.x];
  const int s = w.stamp, ch = blockIdx.y;
  if ((mask && !mask[s]) || skip_ie(mask, s, ch)) return;
  const StampDesc d = desc[s];
  const PathDesc pd = path[s];
  const FftPlan &pl = plans[pd.plan];
  const int L = pl.L, Lh = L / 2 + 1, Ls = L + 1;
  const Geo g = geo_of(MODE, d, L);
  const int T = min(CAP / Ls, tmax);
  float2 *buf = lds, *tw = lds + LDS0;

  int64_t in_base, plane;
  if (MODE == MODE_CONV) { in_base = d.pad; plane = (int64_t)d.Mh * d.Mw; }
  else if (MODE == MODE_CORR) { in_base = d.pix; plane = (int64_t)d.H * d.W; }
  else { in_base = d.psf; plane = (int64_t)d.K * d.K; }
  const float *src = in + in_base * n_ch + ch * plane;
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, (uint32_t)plane * 4u);
  const int r0 = w.unit * 2 * T;
  const FDiv divL(L);
  {
    float va[NIT], vb[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      const int t = divL(idx), n = idx - t * L;
      const int ra = r0 + 2 * t, rb = ra + 1;
      const int c = n - g.in_col0;
      const bool cin = idx < T * L && c >= 0 && c < g.in_cols;
      const bool oka = cin && ra < g.in_rows, okb = cin && rb < g.in_rows;
      va[it] = bload_f32(rsrc, oka ? (uint32_t)(ra * g.in_cols + c) * 4u : kOutOfRange);
      vb[it] = bload_f32(rsrc, okb ? (uint32_t)(rb * g.in_cols + c) * 4u : kOutOfRange);
    }
    stage_twiddles(tw, tw_all + pl.tw_off, L);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      if (idx < T * L) {
        const int t = divL(idx), n = idx - t * L;
        buf[lp(t * Ls + n)] = make_float2(va[it], vb[it]);
      }
    }
  }
  __syncthreads();
  lds_fft<false, RMAX>(buf, T, Ls, pl, tw);
  float2 *dst = S1 + s1_off[s] * n_ch + (int64_t)ch * Lh * g.in_rows;
  const int nr = min(2 * T, g.in_rows - r0);
  const FDiv divNr(nr);
  for (int idx = threadIdx.x; idx < Lh * nr; idx += blockDim.x) {
    const int k = divNr(idx), rr = idx - k * nr;
    const int t = rr >> 1;
    const float2 zk = buf[lp(t * Ls + k)];
    const float2 zc = cconj(buf[lp(t * Ls + (k == 0 ? 0 : L - k))]);
    const float2 v = (rr & 1) ? cscale(mul_mi(csub(zk, zc)), 0.5f) : cscale(cadd(zk, zc), 0.5f);
    dst[(int64_t)k * g.in_rows + r0 + rr] = v;
  }
}

// ---------------------------------------------------------- column pass
// Column k of S1 (rows 0 .. in_rows-1) sits at L-grid rows col_row0 ..;
// MODE_CONV multiplies by the OTF, MODE_CORR by its conjugate, MODE_OTF only
// transforms forward and scales by 1/L^2 (writing the OTF itself, bin-major
// [L/2+1][L]).
template <int MODE, int RMAX>
__global__ __launch_bounds__(kThreads) void k_fft_cols(const StampDesc *__restrict__ desc,
                                                       const PathDesc *__restrict__ path,
                                                       const FftPlan *__restrict__ plans,
                                                       const float2 *__restrict__ tw_all,
                                                       const Work *__restrict__ work, int n_ch,
                                                       const int64_t *__restrict__ s1_off,
                                                       const float2 *__restrict__ S1,
                                                       const float2 *__restrict__ otf,
                                                       const int64_t *__restrict__ s2_off, float2 *__restrict__ S2,
                                                       const int *__restrict__ mask, int tmax, int nx) {
  extern __shared__ float2 lds[];
  constexpr int CAP = fft_cap(RMAX), LDS0 = fft_lds(CAP), NIT = fft_iters(CAP);
  // Workgroup b runs on XCD b % 8 (workgroups go to the eight XCDs in turn);
  // the n_ch channels of one unit take consecutive slots of one XCD, so the
  // unit's OTF block comes from HBM once and from that XCD's L2 for the other
  // channels.  The grid has ceil(nx / 8) * 8 * n_ch workgroups.
  const int xcd = (int)(blockIdx.x & 7u), slot = (int)(blockIdx.x >> 3);
  const int q = slot / n_ch, ch = slot - q * n_ch;
  const int ux = q * 8 + xcd;
  if (ux >= nx) return;
  const Work w = work[ux];
  const int s = w.stamp;
  if ((mask && !mask[s]) || skip_ie(mask, s, ch)) return;
  const StampDesc d = desc[s];
  const PathDesc pd = path[s];
  const FftPlan &pl = plans[pd.plan];
  const int L = pl.L, Lh = L / 2 + 1;
  const Geo g = geo_of(MODE, d, L);
  const int C = min(CAP / L, tmax);
  const int k0 = w.unit * C;
  const int nc = min(C, Lh - k0);
  float2 *buf = lds, *tw = lds + LDS0;

  const float2 *spec = S1 + s1_off[s] * n_ch + (int64_t)ch * Lh * g.in_rows;
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(spec, (uint32_t)(Lh * g.in_rows) * 8u);
  const FDiv divL(L);
  {
    float2 v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      const int c = divL(idx), y = idx - c * L;
      const int r = y - g.col_row0;
      const bool ok = idx < C * L && c < nc && r >= 0 && r < g.in_rows;
      v[it] = bload_f32x2(rsrc, ok ? (uint32_t)((k0 + c) * g.in_rows + r) * 8u : kOutOfRange);
    }
    stage_twiddles(tw, tw_all + pl.tw_off, L);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      if (idx < C * L) buf[lp(idx)] = v[it];
    }
  }
  __syncthreads();
  lds_fft<false, RMAX>(buf, C, L, pl, tw);
  if (MODE == MODE_OTF) {
    const float sc = 1.0f / ((float)L * (float)L);
    float2 *dst = S2 + s2_off[s] + (int64_t)k0 * L;
    for (int idx = threadIdx.x; idx < nc * L; idx += blockDim.x) dst[idx] = cscale(buf[lp(idx)], sc);
    return;
  }
  const __amdgpu_buffer_rsrc_t hrsrc = make_rsrc(otf + pd.otf_mp, (uint32_t)(L * Lh) * 8u);
  {
    float2 hv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      hv[it] = bload_f32x2(hrsrc, idx < nc * L ? (uint32_t)(k0 * L + idx) * 8u : kOutOfRange);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      if (idx < nc * L) {
        const float2 x = buf[lp(idx)];
        buf[lp(idx)] = (MODE == MODE_CORR) ? cmulc(x, hv[it]) : cmul(x, hv[it]);
      }
    }
  }
  __syncthreads();
  lds_fft<true, RMAX>(buf, C, L, pl, tw);
  float2 *dst = S2 + s2_off[s] * n_ch + (int64_t)ch * Lh * g.out_rows + (int64_t)k0 * g.out_rows;
  const FDiv divR(g.out_rows);
  for (int idx = threadIdx.x; idx < nc * g.out_rows; idx += blockDim.x) {
    const int c = divR(idx), y = idx - c * g.out_rows;
    dst[idx] = buf[lp(c * L + g.out_row0 + y)];
  }
}

// ------------------------------------------------------ inverse row pass
// out: stamp s channel ch starts at out_base(s) * n_ch + ch * out_rows * out_cols.
template <int MODE, int RMAX>
__global__ __launch_bounds__(kThreads) void k_fft_irows(const StampDesc *__restrict__ desc,
                                                        const PathDesc *__restrict__ path,
                                                        const FftPlan *__restrict__ plans,
                                                        const float2 *__restrict__ tw_all,
                                                        const Work *__restrict__ work, int n_ch,
                                                        const int64_t *__restrict__ s2_off,
                                                        const float2 *__restrict__ S2, float *__restrict__ out,
                                                        const int *__restrict__ mask, int tmax, Chi2Epi ep) {
  extern __shared__ float2 lds[];
  constexpr int CAP = fft_cap(RMAX), LDS0 = fft_lds(CAP), NIT = fft_iters(CAP);
  const Work w = work[blockIdx.x];
  const int s = w.stamp, ch = blockIdx.y;
  if ((mask && !mask[s]) || skip_ie(mask, s, ch)) return;
  const StampDesc d = desc[s];
  const PathDesc pd = path[s];
  const FftPlan &pl = plans[pd.plan];
  const int L = pl.L, Lh = L / 2 + 1, Ls = L + 1;
  const Geo g = geo_of(MODE, d, L);
  const int T = min(CAP / Ls, tmax);
  float2 *buf = lds, *tw = lds + LDS0;

  const float2 *src = S2 + s2_off[s] * n_ch + (int64_t)ch * Lh * g.out_rows;
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, (uint32_t)(Lh * g.out_rows) * 8u);
  const int r0 = w.unit * 2 * T;
  const FDiv divT(T);
  {
    float2 va[NIT], vb[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      const int k = divT(idx), t = idx - k * T;
      const int ra = r0 + 2 * t, rb = ra + 1;
      const bool ok = idx < T * L;
      const int kk = k > L / 2 ? L - k : k;
      const bool oka = ok && ra < g.out_rows, okb = ok && rb < g.out_rows;
      const uint32_t cb = (uint32_t)(kk * g.out_rows);
      va[it] = bload_f32x2(rsrc, oka ? (cb + (uint32_t)ra) * 8u : kOutOfRange);
      vb[it] = bload_f32x2(rsrc, okb ? (cb + (uint32_t)rb) * 8u : kOutOfRange);
    }
    stage_twiddles(tw, tw_all + pl.tw_off, L);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      if (idx < T * L) {
        const int k = divT(idx), t = idx - k * T;
        float2 A = va[it], B = vb[it];
        if (k > L / 2) {
          A = cconj(A);
          B = cconj(B);
        }
        buf[lp(t * Ls + k)] = cadd(A, mul_i(B));
      }
    }
  }
  __syncthreads();
  lds_fft<true, RMAX>(buf, T, Ls, pl, tw);
  if constexpr (MODE == MODE_CHI2) {
    // w (d - m - sky)^2.  All threads form the squared residuals of
    // the workgroup's rows (every data and weight load in flight at once)
    // and stage them in LDS; then one wave per row pair adds them, lane l
    // taking columns l, l + 64, ... (first row, then second row, at each
    // column), so a pair's partial does not depend on the launch shape.
    const float sky = ep.theta_f64 ? (float)((const double *)ep.theta)[d.par + kNPC * d.ncomp]
                                   : ((const float *)ep.theta)[d.par + kNPC * d.ncomp];
    const uint32_t npix = (uint32_t)(d.H * d.W);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(ep.data + d.img, npix * 4u);
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(ep.weight + d.img, npix * 4u);
    const int oc = g.out_cols, n_items = T * oc;
    const FDiv divO(oc);
    float da[NIT], wa[NIT], db[NIT], wb[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      const int t = divO(idx), x = idx - t * oc;
      const int ra = r0 + 2 * t;
      const bool ina = idx < n_items && ra < g.out_rows, inb = ina && ra + 1 < g.out_rows;
      const uint32_t pa = (uint32_t)(ra * oc + x) * 4u;
      da[it] = bload_f32(rd, ina ? pa : kOutOfRange);
      wa[it] = bload_f32(rw, ina ? pa : kOutOfRange);
      db[it] = bload_f32(rd, inb ? pa + (uint32_t)oc * 4u : kOutOfRange);
      wb[it] = bload_f32(rw, inb ? pa + (uint32_t)oc * 4u : kOutOfRange);
    }
    float2 sq[NIT];
    float *mdst = (ep.model && d.ncomp == 1) ? ep.model + d.pix : nullptr;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      sq[it] = make_float2(0.f, 0.f);
      if (idx < n_items) {
        const int t = divO(idx), x = idx - t * oc;
        const float2 v = buf[lp(t * Ls + g.out_col0 + x)];
        const float ra = da[it] - (v.x + sky), rb = db[it] - (v.y + sky);
        sq[it] = make_float2((wa[it] * ra) * ra, (wb[it] * rb) * rb);   // w r^2: no square root
        if (mdst) {
          const int ra = r0 + 2 * t;
          if (ra < g.out_rows) mdst[(int64_t)ra * oc + x] = v.x;
          if (ra + 1 < g.out_rows) mdst[(int64_t)(ra + 1) * oc + x] = v.y;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = (int)threadIdx.x + it * kThreads;
      if (idx < n_items) buf[idx] = sq[it];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t = wv; t < T; t += kThreads / 64) {
      const int ra = r0 + 2 * t;
      if (ra >= g.out_rows) break;
      const bool hb = ra + 1 < g.out_rows;
      F2 acc = {0.f, 0.f};
      for (int x = lane; x < oc; x += 64) {
        const float2 q = buf[t * oc + x];
        acc = f2_add1(acc, q.x);
        if (hb) acc = f2_add1(acc, q.y);
      }
      acc = wave_sum(acc);
      if (lane == 0) ep.part[ep.first[s] + (ra >> 1)] = make_float2(acc.hi, acc.lo);
    }
    return;
  }
  int64_t out_base = (MODE == MODE_CONV) ? d.pix : d.pad;
  float *dst = out + out_base * n_ch + (int64_t)ch * g.out_rows * g.out_cols;
  const FDiv divC(g.out_cols);
  for (int idx = threadIdx.x; idx < T * g.out_cols; idx += blockDim.x) {
    const int t = divC(idx), x = idx - t * g.out_cols;
    const int ra = r0 + 2 * t, rb = ra + 1;
    const float2 v = buf[lp(t * Ls + g.out_col0 + x)];
    if (ra < g.out_rows) dst[(int64_t)ra * g.out_cols + x] = v.x;
    if (rb < g.out_rows) dst[(int64_t)rb * g.out_cols + x] = v.y;
  }
}

// ----------------------------------------------------------------- launchers
hipError_t launch_fft2d(hipStream_t st, const gf_batch *b, const gf_psf *p, int mode, const float *in, int n_ch,
                        float *out, const int *mask, const WorkView *v, const Chi2Epi *ep,
                        const hipStream_t *bst = nullptr);

static size_t fft_lds_bytes(const gf_psf *p) { return (size_t)(fft_lds(fft_cap(p->rmax)) + p->max_L) * sizeof(float2); }

// Launch the kernel built for the PSF's largest plan radix.
#define GF_FFT_LAUNCH(KERNEL, MODE, ...)                                  \
  do {                                                                   \
    if (p->rmax <= 18)                                                   \
      hipLaunchKernelGGL((KERNEL<MODE, 18>), __VA_ARGS__);               \
    else if (p->rmax <= 24)                                              \
      hipLaunchKernelGGL((KERNEL<MODE, 24>), __VA_ARGS__);               \
    else                                                                 \
      hipLaunchKernelGGL((KERNEL<MODE, 32>), __VA_ARGS__);               \
  } while (0)

// Grid of the column pass for nx work entries of n_ch channels each.
static dim3 cols_grid(int nx, int n_ch) { return dim3((unsigned)((nx + 7) / 8 * 8 * n_ch)); }

// Small jobs (fewer than two workgroups per CU in the wide shape) use the
// narrow shape: one row pair or two bins per workgroup, so more CUs share the
// latency-bound work.
// With ep (one channel only) the inverse-row pass reduces chi^2 partials
// instead of writing out.
static hipError_t multipass_conv(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *in, int n_ch,
                                 float2 *S1, float2 *S2, float *out, const int *mask, const WorkView *v,
                                 const Chi2Epi *ep) {
  const bool view = v && v->rows;
  const int n_cols_w = view ? v->n_cols : (int)p->h_cols.size();
  if ((view ? v->n_rows : (int)p->h_rows.size()) == 0) return hipSuccess;
  const size_t lds = fft_lds_bytes(p);
  dim3 blk(kThreads);
  const bool narrow = (int64_t)n_cols_w * n_ch < 2 * 256;
  const int nr = view ? (narrow ? v->n_rows_n : v->n_rows) : (int)(narrow ? p->h_rows_n : p->h_rows).size();
  const int nc = view ? (narrow ? v->n_cols_n : v->n_cols) : (int)(narrow ? p->h_cols_n : p->h_cols).size();
  const int ni = view ? (narrow ? v->n_irows_n : v->n_irows) : (int)(narrow ? p->h_irows_n : p->h_irows).size();
  const Work *d_rows = view ? (narrow ? v->rows_n : v->rows) : (narrow ? p->d_rows_n : p->d_rows);
  const Work *d_cols = view ? (narrow ? v->cols_n : v->cols) : (narrow ? p->d_cols_n : p->d_cols);
  const Work *d_irows = view ? (narrow ? v->irows_n : v->irows) : (narrow ? p->d_irows_n : p->d_irows);
  const int tr = narrow ? kFftNarrowT : 1 << 20, tc = narrow ? kFftNarrowC : 1 << 20;
  {
    ProfScope ps(st, ep ? "k_fft_rows.chi2" : "k_fft_rows");
    GF_FFT_LAUNCH(k_fft_rows, MODE_CONV, dim3((unsigned)nr, n_ch), blk, lds, st, b->d_desc, p->d_path,
                       p->d_plans, p->d_tw, d_rows, in, n_ch, p->d_s1, S1, mask, tr);
  }
  {
    ProfScope ps(st, ep ? "k_fft_cols.chi2" : "k_fft_cols");
    GF_FFT_LAUNCH(k_fft_cols, MODE_CONV, cols_grid(nc, n_ch), blk, lds, st, b->d_desc, p->d_path, p->d_plans,
                  p->d_tw, d_cols, n_ch, p->d_s1, S1, p->d_otf, p->d_s2, S2, mask, tc, nc);
  }
  {
    ProfScope ps(st, ep ? "k_fft_irows_chi2" : "k_fft_irows");
    if (ep)
      GF_FFT_LAUNCH(k_fft_irows, MODE_CHI2, dim3((unsigned)ni, 1), blk, lds, st, b->d_desc, p->d_path,
                         p->d_plans, p->d_tw, d_irows, 1, p->d_s2, S2, out, mask, tr, *ep);
    else
      GF_FFT_LAUNCH(k_fft_irows, MODE_CONV, dim3((unsigned)ni, n_ch), blk, lds, st, b->d_desc, p->d_path,
                         p->d_plans, p->d_tw, d_irows, n_ch, p->d_s2, S2, out, mask, tr, Chi2Epi{});
  }
  return hipGetLastError();
}

// Every FFT-path stamp of the PSF (or of the view): the one-workgroup
// kernels for the stamps on that form, the three multi-pass launches for the
// rest.  With fork streams and work for more than one of them, the
// one-workgroup buckets run on the side streams (lane kForkLane[b]) beside
// the multi-pass launches (disjoint stamps and outputs) and the caller's
// stream waits for them before anything it runs next; with timing records
// on, everything runs on the caller's stream so that each record times its
// kernels alone.
hipError_t launch_fft_conv(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *in, int n_ch,
                           float2 *S1, float2 *S2, float *out, const int *mask, const WorkView *v,
                           const Chi2Epi *ep, const FftFork *fork) {
  if (ep && n_ch != 1) return hipErrorInvalidValue;
  const int mode = ep ? MODE_CHI2 : MODE_CONV;
  const int *first = (v && v->f2d) ? v->f2d_first : p->f2d_first;
  const bool has_mp = (v && v->rows) ? v->n_rows > 0 : !p->h_rows.empty();
  bool lane_used[kForkLanes] = {};
  int lanes = has_mp ? 1 : 0;
  for (int k = 0; k < kF2dBuckets; ++k)
    if (first[k + 1] > first[k] && !lane_used[kForkLane[k]]) {
      lane_used[kForkLane[k]] = true;
      ++lanes;
    }
  const bool timed = t_prof && t_prof->on;
  if (fork && fork->fork && lanes > 1 && !timed) {
    hipError_t e = hipEventRecord(fork->fork, st);
    for (int i = 0; i < kForkLanes && e == hipSuccess; ++i)
      if (lane_used[i]) e = hipStreamWaitEvent(fork->side[i], fork->fork, 0);
    if (e != hipSuccess) return e;
    hipStream_t bst[kF2dBuckets];
    for (int k = 0; k < kF2dBuckets; ++k) bst[k] = fork->side[kForkLane[k]];
    const hipError_t ef = launch_fft2d(st, b, p, mode, in, n_ch, out, mask, v, ep, bst);
    const hipError_t em = multipass_conv(st, b, p, in, n_ch, S1, S2, out, mask, v, ep);
    // join every forked stream even after a failed launch, so none is left forked
    for (int i = 0; i < kForkLanes; ++i) {
      if (!lane_used[i]) continue;
      hipError_t ej = hipEventRecord(fork->join[i], fork->side[i]);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(st, fork->join[i], 0);
      if (e == hipSuccess) e = ej;
    }
    return ef != hipSuccess ? ef : em != hipSuccess ? em : e;
  }
  hipError_t e = launch_fft2d(st, b, p, mode, in, n_ch, out, mask, v, ep);
  if (e != hipSuccess) return e;
  return multipass_conv(st, b, p, in, n_ch, S1, S2, out, mask, v, ep);
}

hipError_t launch_fft_corr(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *in, float2 *S1,
                           float2 *S2, float *out) {
  hipError_t e = launch_fft2d(st, b, p, MODE_CORR, in, 1, out, nullptr, nullptr, nullptr);
  if (e != hipSuccess) return e;
  if (p->h_arows.empty()) return hipSuccess;
  ProfScope ps(st, "k_fft_corr");
  const size_t lds = fft_lds_bytes(p);
  dim3 blk(kThreads);
  GF_FFT_LAUNCH(k_fft_rows, MODE_CORR, dim3((unsigned)p->h_arows.size(), 1), blk, lds, st, b->d_desc,
                     p->d_path, p->d_plans, p->d_tw, p->d_arows, in, 1, p->d_s1a, S1, (const int *)nullptr, 1 << 20);
  GF_FFT_LAUNCH(k_fft_cols, MODE_CORR, cols_grid((int)p->h_acols.size(), 1), blk, lds, st, b->d_desc,
                     p->d_path, p->d_plans, p->d_tw, p->d_acols, 1, p->d_s1a, S1, p->d_otf, p->d_s2a, S2,
                     (const int *)nullptr, 1 << 20, (int)p->h_acols.size());
  GF_FFT_LAUNCH(k_fft_irows, MODE_CORR, dim3((unsigned)p->h_airows.size(), 1), blk, lds, st, b->d_desc,
                     p->d_path, p->d_plans, p->d_tw, p->d_airows, 1, p->d_s2a, S2, out, (const int *)nullptr,
                     1 << 20, Chi2Epi{});
  return hipGetLastError();
}

// OTF of every FFT stamp: rows of the K x K taps, then forward columns over
// all L rows scaled by 1/L^2.  S1 holds K rows of spectra per stamp.
hipError_t launch_fft_otf(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *taps,
                          const gf::Work *rows, int n_rows, const gf::Work *cols, int n_cols, const int64_t *s1_off,
                          float2 *S1, const int64_t *otf_off) {
  if (n_rows == 0) return hipSuccess;
  const size_t lds = fft_lds_bytes(p);
  dim3 blk(kThreads);
  GF_FFT_LAUNCH(k_fft_rows, MODE_OTF, dim3((unsigned)n_rows, 1), blk, lds, st, b->d_desc, p->d_path,
                     p->d_plans, p->d_tw, rows, taps, 1, s1_off, S1, (const int *)nullptr, 1 << 20);
  GF_FFT_LAUNCH(k_fft_cols, MODE_OTF, cols_grid(n_cols, 1), blk, lds, st, b->d_desc, p->d_path,
                     p->d_plans, p->d_tw, cols, 1, s1_off, S1, (const float2 *)nullptr, otf_off, p->d_otf,
                     (const int *)nullptr, 1 << 20, n_cols);
  return hipGetLastError();
}

}  // namespace gf

// fft2d_impl.h -- step 2 of the fitting loop (Barsdell et al., Sec. 3 item 2:
// FFT plus a pointwise transform) for FFT sides up to 192, one workgroup per
// stamp and channel, with the whole 2-D half spectrum held in LDS.
//
// Sec. 3 observes that a 2-D FFT is an all-to-all step; on this chip an
// L x (L/2 + 1) complex half spectrum with L <= 192 fits in one workgroup's
// 160 KB of LDS, so the all-to-all stays on chip and the only HBM traffic of
// a convolution is the padded model read once, the OTF read once and the
// H x W result written once (or, for the chi^2 epilogue, the observation and
// weights read once).  The layout in LDS is row-major, rows of L/2 + 1 bins:
//   1. rows, two real rows per complex transform z = a + i b, each transform
//      done in place over its row pair's 2 (L/2 + 1) >= L slots;
//   2. split each row pair's spectrum into the two half spectra A, B (rows
//      2t and 2t + 1 of the layout);
//   3. columns: L/2 + 1 transforms of stride L/2 + 1, times the OTF (stored
//      row-major [L][L/2 + 1] for this path, so its loads are contiguous),
//      inverse transforms;
//   4. the kept rows rebuilt pairwise as Z = A + i B over all L bins
//      (Hermitian symmetry for the upper half), inverse transforms, real part
//      to the first row and imaginary part to the second, crop.
// One extra row of slack lets the last row pair's transform run past row
// L - 1.  The 1/L^2 of the inverse transform is folded into the OTF.
//
// The transform side, its radix plan, the thread count and the loop bounds
// are compile-time constants of each kernel; every index division is by a
// constant.  Loads of the input, the OTF, the observation and the weights
// go through range-checked buffer resources, as in the multi-pass kernels.
#pragma once

#include "gf_internal.h"
#include "bufload.h"
#include "fft_dft.h"
#include "twosum.h"

namespace gf {
namespace {

// LDS index with one padding slot per 32 complex values (spreads the
// strided Stockham stores over the banks).
__device__ __forceinline__ int lq(int i) { return i + (i >> 5); }
constexpr int lq_size(int n) { return n + n / 32 + 1; }

// Radices of the LDS passes for side L: one pass when L is itself a radix of
// at most 16, otherwise the two-factor split with the smallest larger factor
// (the busiest thread's register count), radices up to 18.
constexpr bool f2_radix(int r) {
  return r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 8 || r == 9 || r == 10 || r == 12 || r == 15 ||
         r == 16 || r == 18;
}
struct F2Plan {
  int n, r0, r1;
};
constexpr F2Plan f2_plan(int L) {
  if (L <= 16 && f2_radix(L)) return F2Plan{1, L, 1};
  F2Plan best{0, 0, 0};
  for (int a = 2; a <= 18; ++a) {
    if (!f2_radix(a) || L % a) continue;
    const int b = L / a;
    if (!f2_radix(b) || b > a) continue;
    if (best.n == 0 || a < best.r0) best = F2Plan{2, a, b};
  }
  return best;
}

constexpr int f2_lds_bytes(int L) { return (lq_size((L + 1) * (L / 2 + 1)) + L) * 8; }
// Threads per workgroup: enough for about 16 waves per CU at the number of
// workgroups the LDS allows.
constexpr int f2_threads(int L) {
  const int wg = (160 * 1024) / f2_lds_bytes(L);
  return wg >= 4 ? 256 : wg >= 2 ? 512 : 1024;
}
// Largest side of bucket B, whose LDS and thread count its kernel is built for.
constexpr int f2b_maxL(int B) { return kF2dSides[kF2dBucketEnd[B] - 1]; }
constexpr int f2b_first(int B) { return B == 0 ? 0 : kF2dBucketEnd[B - 1]; }

// One Stockham pass of radix R over ntr transforms of length L in place.
// Element n of a row transform t sits at row0 LH + 2 t LH + n (its row
// pair's slots); element n of column transform k at n LH + k.  Every thread
// first loads and computes all of its butterflies, the workgroup
// synchronises, then all results are stored.
template <int L, int R, int NS, bool INV, int NT, int TMAX, bool COLS>
__device__ __forceinline__ void f2_pass(float2 *__restrict__ buf, const float2 *__restrict__ tw, int ntr, int row0) {
  constexpr int LH = L / 2 + 1;
  constexpr int NBF = L / R;
  constexpr int STRIDE = COLS ? LH : 1;
  constexpr int NB = (TMAX * NBF + NT - 1) / NT;
  const int total = ntr * NBF;
  float2 v[NB][R];
  int dst[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int q = (int)threadIdx.x + b * NT;
    dst[b] = -1;
    if (q < total) {
      int base, j;
      if (COLS) {
        const int k = q % LH;
        j = q / LH;
        base = k;
      } else {
        const int t = q / NBF;
        j = q - t * NBF;
        base = (row0 + 2 * t) * LH;
      }
      const int kk = j % NS, jd = j / NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[lq(base + (j + r * NBF) * STRIDE)];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[r * kk * (L / (NS * R))];
          v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
        }
      }
      dft<R, INV>(v[b]);
      dst[b] = base + (jd * NS * R + kk) * STRIDE;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (dst[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lq(dst[b] + r * NS * STRIDE)] = v[b][r];
    }
  }
  __syncthreads();
}

template <int L, bool INV, int NT, int TMAX, bool COLS>
__device__ __forceinline__ void f2_fft(float2 *buf, const float2 *tw, int ntr, int row0) {
  constexpr F2Plan pl = f2_plan(L);
  static_assert(pl.n == 1 || pl.n == 2, "no plan for this side");
  if constexpr (pl.n == 1) {
    f2_pass<L, pl.r0, 1, INV, NT, TMAX, COLS>(buf, tw, ntr, row0);
  } else {
    f2_pass<L, pl.r0, 1, INV, NT, TMAX, COLS>(buf, tw, ntr, row0);
    f2_pass<L, pl.r1, pl.r0, INV, NT, TMAX, COLS>(buf, tw, ntr, row0);
  }
}

// Division by a value fixed for the workgroup (x, d < 2^16).
struct Div16 {
  uint32_t m;
  __device__ __forceinline__ explicit Div16(int d) : m(d <= 1 ? 0u : 0xffffffffu / (uint32_t)d + 1u) {}
  __device__ __forceinline__ int operator()(int x) const { return m ? (int)__umulhi((uint32_t)x, m) : x; }
};

}  // namespace

// The convolution of one (stamp, channel) of side L by a workgroup of NT
// threads, in the LDS buffers buf (lq_size((L + 1)(L/2 + 1)) values) and tw
// (L values).
template <int L, int MODE, int NT>
__device__ __forceinline__ void f2_body(float2 *__restrict__ buf, float2 *__restrict__ tw, const StampDesc &d,
                                        const PathDesc &pd, int s, int ch, const float2 *__restrict__ tw_all,
                                        const float *__restrict__ in, int n_ch, float *__restrict__ out,
                                        const float2 *__restrict__ otf, float2 *__restrict__ otf_out,
                                        const Chi2Epi &ep) {
  constexpr int LH = L / 2 + 1;
  const float2 *twl = tw_all + pd.tw;
  const int tid = (int)threadIdx.x;
  const int km1 = d.K - 1;

  // geometry of the mode
  int in_rows, in_cols, row0, out_row0, out_rows, out_col0, out_cols;
  const float *src;
  if (MODE == MODE_CONV || MODE == MODE_CHI2) {
    in_rows = d.Mh; in_cols = d.Mw; row0 = 0;
    out_row0 = km1; out_rows = d.H; out_col0 = km1; out_cols = d.W;
    src = in + d.pad * n_ch + (int64_t)ch * d.Mh * d.Mw;
  } else if (MODE == MODE_CORR) {
    in_rows = d.H; in_cols = d.W; row0 = km1;
    out_row0 = 0; out_rows = d.Mh; out_col0 = 0; out_cols = d.Mw;
    src = in + d.pix * n_ch + (int64_t)ch * d.H * d.W;
  } else {
    in_rows = d.K; in_cols = d.K; row0 = 0;
    out_row0 = 0; out_rows = L; out_col0 = 0; out_cols = 0;
    src = in + d.psf;
  }
  const int col0 = row0;

  // ---- 1. load the input row pairs (zero outside the input), twiddles
  const int rows_end = row0 + in_rows;
  const int P = (rows_end + 1) >> 1;
  {
    constexpr int NI = ((L / 2) * L + NT - 1) / NT;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, (uint32_t)(in_rows * in_cols) * 4u);
    float va[NI], vb[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      const int t = q / L, n = q - t * L;
      const int ra = 2 * t - row0, c = n - col0;
      const bool ok = q < P * L && c >= 0 && c < in_cols;
      const bool oka = ok && ra >= 0 && ra < in_rows, okb = ok && ra + 1 >= 0 && ra + 1 < in_rows;
      va[it] = bload_f32(rs, oka ? (uint32_t)(ra * in_cols + c) * 4u : kOutOfRange);
      vb[it] = bload_f32(rs, okb ? (uint32_t)((ra + 1) * in_cols + c) * 4u : kOutOfRange);
    }
    {
      const __amdgpu_buffer_rsrc_t rt = make_rsrc(twl, (uint32_t)L * 8u);
      for (int i = tid; i < L; i += NT) tw[i] = bload_f32x2(rt, (uint32_t)i * 8u);
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      if (q < P * L) {
        const int t = q / L, n = q - t * L;
        buf[lq(2 * t * LH + n)] = make_float2(va[it], vb[it]);
      }
    }
    // rows 2P .. L-1 of the half spectrum are zero
    for (int i = 2 * P * LH + tid; i < L * LH; i += NT) buf[lq(i)] = make_float2(0.f, 0.f);
  }
  __syncthreads();

  // ---- 2. row transforms, then the split into the half spectra A, B
  f2_fft<L, false, NT, L / 2, false>(buf, tw, P, 0);
  {
    constexpr int NI = ((L / 2) * LH + NT - 1) / NT;
    float2 A[NI], B[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      if (q < P * LH) {
        const int t = q / LH, k = q - t * LH;
        const float2 zk = buf[lq(2 * t * LH + k)];
        const float2 zc = cconj(buf[lq(2 * t * LH + (k == 0 ? 0 : L - k))]);
        A[it] = cscale(cadd(zk, zc), 0.5f);
        B[it] = cscale(mul_mi(csub(zk, zc)), 0.5f);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      if (q < P * LH) {
        const int t = q / LH, k = q - t * LH;
        buf[lq(2 * t * LH + k)] = A[it];
        buf[lq((2 * t + 1) * LH + k)] = B[it];
      }
    }
  }
  __syncthreads();

  // ---- 3. column transforms, OTF product, inverse column transforms
  f2_fft<L, false, NT, LH, true>(buf, tw, LH, 0);
  constexpr int NIO = (L * LH + NT - 1) / NT;
  if constexpr (MODE == MODE_OTF) {
    const float sc = 1.0f / ((float)L * (float)L);
    float2 *dst = otf_out + pd.otf;
#pragma unroll
    for (int it = 0; it < NIO; ++it) {
      const int q = tid + it * NT;
      if (q < L * LH) dst[q] = cscale(buf[lq(q)], sc);
    }
    return;
  } else {
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(otf + pd.otf, (uint32_t)(L * LH) * 8u);
    float2 h[NIO];
#pragma unroll
    for (int it = 0; it < NIO; ++it) h[it] = bload_f32x2(ro, (uint32_t)(tid + it * NT) * 8u);
#pragma unroll
    for (int it = 0; it < NIO; ++it) {
      const int q = tid + it * NT;
      if (q < L * LH) {
        const float2 x = buf[lq(q)];
        buf[lq(q)] = (MODE == MODE_CORR) ? cmulc(x, h[it]) : cmul(x, h[it]);
      }
    }
  }
  __syncthreads();
  f2_fft<L, true, NT, LH, true>(buf, tw, LH, 0);

  // ---- 4. kept rows pairwise: Z = A + i B over all L bins, inverse rows
  const int Q = (out_rows + 1) >> 1;
  {
    constexpr int NI = ((L / 2) * L + NT - 1) / NT;
    float2 Z[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      if (q < Q * L) {
        const int t = q / L, k = q - t * L;
        const int ra = out_row0 + 2 * t;
        const int kk = k <= L / 2 ? k : L - k;
        float2 A = buf[lq(ra * LH + kk)];
        float2 B = (2 * t + 1 < out_rows) ? buf[lq((ra + 1) * LH + kk)] : make_float2(0.f, 0.f);
        if (k > L / 2) {
          A = cconj(A);
          B = cconj(B);
        }
        Z[it] = cadd(A, mul_i(B));
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      if (q < Q * L) {
        const int t = q / L, k = q - t * L;
        buf[lq((out_row0 + 2 * t) * LH + k)] = Z[it];
      }
    }
  }
  __syncthreads();
  f2_fft<L, true, NT, L / 2, false>(buf, tw, Q, out_row0);

  // ---- 5. output rows (crop), or the chi^2 epilogue
  const int oc = out_cols;
  if constexpr (MODE == MODE_CHI2) {
    // w (d - m - sky)^2; one wave per output row pair, lane l taking
    // columns l, l + 64, ... (first row, then second row, at each column),
    // compensated, then summed across the wave: the partial of a pair is
    // the one the multi-pass inverse-row kernel forms.  The next pair's
    // observation and weights are loaded before the current pair is summed.
    constexpr int NCOL = (L + 63) / 64;
    const float sky = ep.theta_f64 ? (float)((const double *)ep.theta)[d.par + kNPC * d.ncomp]
                                   : ((const float *)ep.theta)[d.par + kNPC * d.ncomp];
    const uint32_t npix = (uint32_t)(d.H * d.W);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(ep.data + d.img, npix * 4u);
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(ep.weight + d.img, npix * 4u);
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NW = NT / 64;
    float da[NCOL], wa[NCOL], db[NCOL], wb[NCOL];
    float *mdst = (ep.model && d.ncomp == 1) ? ep.model + d.pix : nullptr;
    auto fetch = [&](int t) {
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        const int x = lane + 64 * c;
        const bool ina = t < Q && x < oc, inb = ina && 2 * t + 1 < out_rows;
        const uint32_t pa = (uint32_t)(2 * t * oc + x) * 4u;
        da[c] = bload_f32(rd, ina ? pa : kOutOfRange);
        wa[c] = bload_f32(rw, ina ? pa : kOutOfRange);
        db[c] = bload_f32(rd, inb ? pa + (uint32_t)oc * 4u : kOutOfRange);
        wb[c] = bload_f32(rw, inb ? pa + (uint32_t)oc * 4u : kOutOfRange);
      }
    };
    fetch(wv);
    for (int t = wv; t < Q; t += NW) {
      float ea[NCOL], eb[NCOL];
      const bool hb = 2 * t + 1 < out_rows;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        const int x = lane + 64 * c;
        ea[c] = 0.f;
        eb[c] = 0.f;
        if (x < oc) {
          const float2 v = buf[lq((out_row0 + 2 * t) * LH + out_col0 + x)];
          const float ra = da[c] - (v.x + sky), rb = db[c] - (v.y + sky);
          ea[c] = (wa[c] * ra) * ra;   // w r^2: no square root
          eb[c] = (wb[c] * rb) * rb;
          if (mdst) {
            mdst[(int64_t)(2 * t) * oc + x] = v.x;
            if (hb) mdst[(int64_t)(2 * t + 1) * oc + x] = v.y;
          }
        }
      }
      fetch(t + NW);
      F2 acc = {0.f, 0.f};
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        if (lane + 64 * c < oc) {
          acc = f2_add1(acc, ea[c]);
          if (hb) acc = f2_add1(acc, eb[c]);
        }
      }
      acc = wave_sum(acc);
      if (lane == 0) ep.part[ep.first[s] + t] = make_float2(acc.hi, acc.lo);
    }
  } else {
    const int64_t out_base = (MODE == MODE_CONV) ? d.pix : d.pad;
    float *dst = out + out_base * n_ch + (int64_t)ch * out_rows * oc;
    const Div16 divc(oc);
    for (int q = tid; q < Q * oc; q += NT) {
      const int t = divc(q), x = q - t * oc;
      const float2 v = buf[lq((out_row0 + 2 * t) * LH + out_col0 + x)];
      dst[(int64_t)(2 * t) * oc + x] = v.x;
      if (2 * t + 1 < out_rows) dst[(int64_t)(2 * t + 1) * oc + x] = v.y;
    }
  }
}

// Dispatch on the stamp's side among the classes I .. HI - 1 of a bucket.
template <int MODE, int NT, int I, int HI>
__device__ __forceinline__ void f2_dispatch(int L, float2 *buf, float2 *tw, const StampDesc &d, const PathDesc &pd,
                                            int s, int ch, const float2 *tw_all, const float *in, int n_ch,
                                            float *out, const float2 *otf, float2 *otf_out, const Chi2Epi &ep) {
  if constexpr (I < HI) {
    if (L == kF2dSides[I])
      f2_body<kF2dSides[I], MODE, NT>(buf, tw, d, pd, s, ch, tw_all, in, n_ch, out, otf, otf_out, ep);
    else
      f2_dispatch<MODE, NT, I + 1, HI>(L, buf, tw, d, pd, s, ch, tw_all, in, n_ch, out, otf, otf_out, ep);
  }
}

// One workgroup per (list entry, channel) of the stamps of bucket B (sides
// kF2dSides[f2b_first(B)] .. f2b_maxL(B)); the LDS and thread count are the
// bucket's largest side's.  Workgroup ids are assigned so that the n_ch
// channels of a stamp get ids equal mod 8, which places them on one XCD,
// where they share the L2 copy of their OTF.
template <int B, int MODE>
__global__ __launch_bounds__(f2_threads(f2b_maxL(B))) void k_fft2d(const StampDesc *__restrict__ desc,
                                                                   const PathDesc *__restrict__ path,
                                                                   const float2 *__restrict__ tw_all,
                                                                   const Work *__restrict__ list, int n_list,
                                                                   const float *__restrict__ in, int n_ch,
                                                                   float *__restrict__ out,
                                                                   const float2 *__restrict__ otf,
                                                                   float2 *__restrict__ otf_out,
                                                                   const int *__restrict__ mask, Chi2Epi ep) {
  constexpr int LM = f2b_maxL(B), NT = f2_threads(LM);
  __shared__ float2 buf[lq_size((LM + 1) * (LM / 2 + 1))];
  __shared__ float2 tw[LM];
  const int blk = (int)blockIdx.x;
  const int grp = blk / (8 * n_ch), rem = blk - grp * 8 * n_ch;
  const int ch = rem >> 3, li = grp * 8 + (rem & 7);
  if (li >= n_list) return;
  const int s = list[li].stamp;
  if ((mask && !mask[s]) || skip_ie(mask, s, ch)) return;
  const StampDesc d = desc[s];
  const PathDesc pd = path[s];
  f2_dispatch<MODE, NT, f2b_first(B), kF2dBucketEnd[B]>(pd.L, buf, tw, d, pd, s, ch, tw_all, in, n_ch, out, otf,
                                                        otf_out, ep);
}

// Launch bucket B's kernel over its n list entries.
template <int B>
hipError_t f2_launch_bucket(int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc, const PathDesc *path,
                            const float2 *tw_all, const Work *list, const float *in, float *out, const float2 *otf,
                            float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  const unsigned blocks = (unsigned)(((n + 7) / 8) * 8 * n_ch);
  const dim3 grid(blocks), block(f2_threads(f2b_maxL(B)));
  switch (mode) {
    case MODE_CONV:
      hipLaunchKernelGGL((k_fft2d<B, MODE_CONV>), grid, block, 0, st, desc, path, tw_all, list, n, in, n_ch, out,
                         otf, otf_out, mask, ep);
      break;
    case MODE_CORR:
      hipLaunchKernelGGL((k_fft2d<B, MODE_CORR>), grid, block, 0, st, desc, path, tw_all, list, n, in, n_ch, out,
                         otf, otf_out, mask, ep);
      break;
    case MODE_OTF:
      hipLaunchKernelGGL((k_fft2d<B, MODE_OTF>), grid, block, 0, st, desc, path, tw_all, list, n, in, n_ch, out,
                         otf, otf_out, mask, ep);
      break;
    default:
      hipLaunchKernelGGL((k_fft2d<B, MODE_CHI2>), grid, block, 0, st, desc, path, tw_all, list, n, in, n_ch, out,
                         otf, otf_out, mask, ep);
      break;
  }
  return hipGetLastError();
}

hipError_t f2d_launch_b0(int, hipStream_t, int, int, const StampDesc *, const PathDesc *, const float2 *,
                         const Work *, const float *, float *, const float2 *, float2 *, const int *, const Chi2Epi &);
hipError_t f2d_launch_b1(int, hipStream_t, int, int, const StampDesc *, const PathDesc *, const float2 *,
                         const Work *, const float *, float *, const float2 *, float2 *, const int *, const Chi2Epi &);
hipError_t f2d_launch_b2(int, hipStream_t, int, int, const StampDesc *, const PathDesc *, const float2 *,
                         const Work *, const float *, float *, const float2 *, float2 *, const int *, const Chi2Epi &);
hipError_t f2d_launch_b3(int, hipStream_t, int, int, const StampDesc *, const PathDesc *, const float2 *,
                         const Work *, const float *, float *, const float2 *, float2 *, const int *, const Chi2Epi &);
hipError_t f2d_launch_b4(int, hipStream_t, int, int, const StampDesc *, const PathDesc *, const float2 *,
                         const Work *, const float *, float *, const float2 *, float2 *, const int *, const Chi2Epi &);

}  // namespace gf

// k_direct.hip -- step 2 of the fitting loop as a direct sum over PSF taps
// for small PSFs (Barsdell et al., Sec. 2 step 2), LDS-tiled for gfx950.
//
// A workgroup computes a 16 x 64 output tile.  The input tile with its
// (K-1)-pixel halo and the K x K taps are staged in LDS; each thread owns one
// output column and four consecutive output rows, so every LDS input value
// it loads feeds up to four accumulators.
//   MODE_CONV:  out[y][x] = sum_{a,b} P[K-1-a][K-1-b] in[y+a][x+b]   (H x W from Mh x Mw)
//   MODE_CORR:  out[y][x] = sum_{a,b} P[a][b] in[y+a-(K-1)][x+b-(K-1)] (Mh x Mw from H x W, zero outside)
// The second is the transpose of the first (the adjoint of the PSF blur).
#include "gf_internal.h"
#include "bufload.h"

namespace gf {

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_direct(const StampDesc *__restrict__ desc,
                                                     const Work *__restrict__ work, const float *__restrict__ in,
                                                     int n_ch, const float *__restrict__ taps,
                                                     float *__restrict__ out, const int *__restrict__ mask) {
  extern __shared__ float smem[];
  const Work w = work[blockIdx.x];
  const int s = w.stamp, ch = blockIdx.y;
  if ((mask && !mask[s]) || skip_ie(mask, s, ch)) return;
  const StampDesc d = desc[s];
  const int K = d.K;
  const int Hout = MODE == 0 ? d.H : d.Mh, Wout = MODE == 0 ? d.W : d.Mw;
  const int Hin = MODE == 0 ? d.Mh : d.H, Win = MODE == 0 ? d.Mw : d.W;
  const int off = MODE == 0 ? 0 : -(K - 1);
  const int tiles_x = (Wout + kDirectTW - 1) / kDirectTW;
  const int ty = w.unit / tiles_x, tx = w.unit - ty * tiles_x;
  const int y0 = ty * kDirectTH, x0 = tx * kDirectTW;
  const int TWp = kDirectTW + K - 1, THp = kDirectTH + K - 1;
  float *F = smem;               // K*K taps, flipped for MODE_CONV
  float *tile = smem + K * K;    // THp x TWp
  // Staging: batches of 8 range-checked loads per thread, all in flight
  // before the LDS stores (out-of-image halo pixels read zero).
  const __amdgpu_buffer_rsrc_t prs = make_rsrc(taps + d.psf, (uint32_t)(K * K) * 4u);
  for (int i0 = 0; i0 < K * K; i0 += 8 * kThreads) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kThreads + (int)threadIdx.x;
      const int a = i / K, b = i - a * K;
      const int src = MODE == 0 ? (K - 1 - a) * K + (K - 1 - b) : i;
      v[q] = bload_f32(prs, i < K * K ? (uint32_t)src * 4u : kOutOfRange);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kThreads + (int)threadIdx.x;
      if (i < K * K) F[i] = v[q];
    }
  }
  const int64_t ibase = (MODE == 0 ? d.pad : d.pix) * (int64_t)n_ch + (int64_t)ch * Hin * Win;
  const __amdgpu_buffer_rsrc_t irs = make_rsrc(in + ibase, (uint32_t)(Hin * Win) * 4u);
  for (int i0 = 0; i0 < THp * TWp; i0 += 8 * kThreads) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kThreads + (int)threadIdx.x;
      const int r = i / TWp, c = i - r * TWp;
      const int yy = y0 + r + off, xx = x0 + c + off;
      const bool ok = i < THp * TWp && yy >= 0 && yy < Hin && xx >= 0 && xx < Win;
      v[q] = bload_f32(irs, ok ? (uint32_t)(yy * Win + xx) * 4u : kOutOfRange);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kThreads + (int)threadIdx.x;
      if (i < THp * TWp) tile[i] = v[q];
    }
  }
  __syncthreads();
  const int x = threadIdx.x & (kDirectTW - 1);
  const int rg = (threadIdx.x / kDirectTW) * 4;   // first of four output rows of this thread
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  // output row rg+o uses input rows rg+o .. rg+o+K-1 (tile coordinates)
  for (int ri = 0; ri < K + 3; ++ri) {
    const float *trow = tile + (rg + ri) * TWp + x;
#pragma unroll 4
    for (int b = 0; b < K; ++b) {
      const float v = trow[b];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int a = ri - o;
        if (a >= 0 && a < K) acc[o] = fmaf(F[a * K + b], v, acc[o]);
      }
    }
  }
  const int64_t obase = (MODE == 0 ? d.pix : d.pad) * (int64_t)n_ch + (int64_t)ch * Hout * Wout;
  const int xo = x0 + x;
  if (xo < Wout) {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int yo = y0 + rg + o;
      if (yo < Hout) out[obase + (int64_t)yo * Wout + xo] = acc[o];
    }
  }
}

static size_t direct_lds_bytes(int K) {
  return (size_t)(K * K + (kDirectTH + K - 1) * (kDirectTW + K - 1)) * sizeof(float);
}

hipError_t launch_direct(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *in, int n_ch, float *out,
                         bool corr, const int *mask, const WorkView *v) {
  const bool view = !corr && v && v->rows;   // a view always carries a direct list (possibly empty)
  const int nlst = view ? v->n_direct : (int)(corr ? p->h_adirect : p->h_direct).size();
  if (nlst == 0) return hipSuccess;
  int maxK = 1;
  for (const auto &d : b->h_desc) maxK = d.K > maxK ? d.K : maxK;
  const size_t lds = direct_lds_bytes(maxK);
  ProfScope ps(st, corr ? "k_direct_corr" : "k_direct");
  if (corr)
    hipLaunchKernelGGL((k_direct<1>), dim3((unsigned)nlst, n_ch), dim3(kThreads), lds, st, b->d_desc,
                       p->d_adirect, in, n_ch, p->d_taps, out, mask);
  else
    hipLaunchKernelGGL((k_direct<0>), dim3((unsigned)nlst, n_ch), dim3(kThreads), lds, st, b->d_desc,
                       view ? v->direct : p->d_direct, in, n_ch, p->d_taps, out, mask);
  return hipGetLastError();
}

}  // namespace gf

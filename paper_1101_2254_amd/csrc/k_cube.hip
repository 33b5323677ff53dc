// k_cube.hip -- kernels of the data-cube path: the model cube and its
// derivatives on the padded grid (step 1 in three dimensions), the spectral
// convolution with the line-spread function, the continuum, the Jacobian
// assembly and the start-point clip.  The spatial convolution of every
// channel, chi^2, the normal equations and the LM state use the image
// kernels through the batches that cube_api.cpp builds.
//
// Model (Sec. 5 names cube fitting as the next use of the three steps; the
// model is a reading): the light of one Sersic component carries a Gaussian
// line centred at the line-of-sight velocity of a thin rotating disk with
// the component's geometry,
//   V = v0 + vproj (2/pi) atan(R/rt) x'/R   (v0 at R = 0),
// and a voxel is the mean over S x S spatial and Sv spectral sub-samples of
// I exp(-(v - V)^2 / (2 sigma^2)).
#include "comp.h"
#include "gf_internal.h"

namespace gf {

namespace {

constexpr float kTwoOverPi = 0.63661977236758134f;
constexpr float kLog2e = 1.4426950408889634f;

// Kinematic constants of a cube.
struct Kin {
  float v0, kv, rt, irt, kg, is2, isg;
};

__device__ __forceinline__ Kin kin_setup(const double *t) {
  Kin k;
  k.v0 = (float)t[8];
  k.kv = (float)t[9] * kTwoOverPi;           // vproj 2/pi
  k.rt = (float)t[10];
  k.irt = 1.0f / k.rt;
  const float sg = (float)t[11];
  k.is2 = 1.0f / (sg * sg);
  k.isg = 1.0f / sg;
  k.kg = -0.5f * kLog2e * k.is2;             // exp(-u^2 / (2 sigma^2)) = exp2(kg u^2)
  return k;
}

// atan(R/rt)/R (1/rt at R = 0).
__device__ __forceinline__ float f_of_r(float R, const Kin &k) {
  return R > 0.0f ? atanf(R * k.irt) / R : k.irt;
}

// f'(R)/R = (R rt/(rt^2 + R^2) - atan(R/rt)) / R^3, by its Taylor series in
// z = R/rt below z = 0.3 (the direct form cancels there), -2/(3 rt^3) at 0:
// rt^3 f'/R = sum_k (-1)^k 2k/(2k+1) z^(2k-2).
__device__ __forceinline__ float g_of_r(float R, const Kin &k) {
  const float z = R * k.irt;
  const float irt3 = k.irt * k.irt * k.irt;
  if (z < 0.3f) {
    const float z2 = z * z;
    float p = 12.0f / 13.0f;
    p = fmaf(p, z2, -10.0f / 11.0f);
    p = fmaf(p, z2, 8.0f / 9.0f);
    p = fmaf(p, z2, -6.0f / 7.0f);
    p = fmaf(p, z2, 4.0f / 5.0f);
    p = fmaf(p, z2, -2.0f / 3.0f);
    return p * irt3;
  }
  return (z / (1.0f + z * z) - atanf(z)) / (R * R * R);
}

// Spectral sub-sample offsets ((2t + 1 - Sv) / (2 Sv)).
__device__ __forceinline__ float sv_off(int t, int Sv) { return (float)(2 * t + 1 - Sv) / (float)(2 * Sv); }

}  // namespace

// Model cube on the padded grid: out[pad * Mc + pc * Mh*Mw + p].  One thread
// per padded spaxel keeps the S^2 sub-samples' intensity and velocity in
// registers and walks the Mc padded channels (each channel plane is written
// by consecutive threads).
template <int S>
__global__ __launch_bounds__(kThreads) void k_cube_eval(const CubeDesc *__restrict__ desc, const Work *__restrict__ work,
                                                        const double *__restrict__ theta, const float4 *__restrict__ bn,
                                                        int Nc, int Kl, int Sv, const int *__restrict__ mask,
                                                        float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const CubeDesc d = desc[s];
  const int np = d.Mh * d.Mw;
  const int p = w.unit * kThreads + (int)threadIdx.x;
  if (p >= np) return;
  const int Mc = Nc + Kl - 1, cl = (Kl - 1) >> 1, c0 = (d.K - 1) >> 1;
  const int pi = p / d.Mw, pj = p - pi * d.Mw;
  const double *t = theta + d.par;
  CompC C;
  comp_setup<double>(t, bn, S, C);
  const Kin k = kin_setup(t);
  const float jx = (float)(pj - c0 - C.ix), iy = (float)(pi - c0 - C.iy);
  const float peak = C.lie + C.b1;
  float I[S * S], V[S * S];
#pragma unroll
  for (int b = 0; b < S; ++b) {
    const float dy = iy + C.oy[b];
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const float dx = jx + C.ox[a];
      const float xp = fmaf(dx, C.cs, dy * C.sn);
      const float yq = fmaf(-dx, C.sq, dy * C.cq);
      const float r2 = fmaf(yq, yq, xp * xp);
      const float tt = fast_exp2(fmaf(fast_log2(r2), C.a1, C.a0));
      I[b * S + a] = fast_exp2(fmaf(-C.b1, tt, peak));
      V[b * S + a] = fmaf(k.kv * xp, f_of_r(sqrtf(r2), k), k.v0);
    }
  }
  const float inv = 1.0f / (float)(S * S * Sv);
  float *dst = out + d.pad * (int64_t)Mc + p;
  for (int pc = 0; pc < Mc; ++pc) {
    const float vb = (float)(pc - cl);
    float acc = 0.0f;
    for (int tv = 0; tv < Sv; ++tv) {
      const float v = vb + sv_off(tv, Sv);
#pragma unroll
      for (int q = 0; q < S * S; ++q) {
        const float u = v - V[q];
        acc = fmaf(I[q], fast_exp2(k.kg * u * u), acc);
      }
    }
    dst[(int64_t)pc * np] = acc * inv;
  }
}

// Derivatives of the model cube on the padded grid, 11 channels (every
// parameter but the continuum, in parameter order):
// out[pad * Mc * 11 + (j * Mc + pc) * Mh*Mw + p].  Per sub-sample the value
// is I G with G = exp(-(v - V)^2 / (2 sigma^2)), so
//   d/dtheta = (dI/dtheta) G + I (dV/dtheta) G (v - V)/sigma^2,
//   d/dsigma = (I/sigma) G (v - V)^2/sigma^2.
// Sersic terms as the image Jacobian (with u = R/Re, t = u^(1/n), E = b_n t:
// dI/dRe = I E/(n Re), dI/dn = I (b'_n (1 - t) + E ln u/n^2),
// dI/dR = -I E/(n R), zero at R = 0 for the 1/R and ln u terms); with
// R dR = x' dx' + (y'/q^2) dy' per geometric parameter and f = atan(R/rt)/R,
//   dV/dtheta = (2/pi) vproj (f dx'/dtheta + x' (f'/R) R dR/dtheta),
//   dV/dvproj = (2/pi) x' f,  dV/drt = -(2/pi) vproj x'/(rt^2 + R^2).
// The channels are taken in blocks of CB; each block recomputes the
// sub-samples' coefficients and keeps 11 CB sums in registers.
#ifndef GF_CUBE_CB
#define GF_CUBE_CB 12
#endif
constexpr int kCubeCB = GF_CUBE_CB;

template <int S>
__global__ __launch_bounds__(kThreads) void k_cube_jac(const CubeDesc *__restrict__ desc, const Work *__restrict__ work,
                                                       const double *__restrict__ theta, const float4 *__restrict__ bn,
                                                       int Nc, int Kl, int Sv, const int *__restrict__ mask,
                                                       float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const CubeDesc d = desc[s];
  const int np = d.Mh * d.Mw;
  const int p = w.unit * kThreads + (int)threadIdx.x;
  if (p >= np) return;
  const int Mc = Nc + Kl - 1, cl = (Kl - 1) >> 1, c0 = (d.K - 1) >> 1;
  const int pi = p / d.Mw, pj = p - pi * d.Mw;
  const double *t = theta + d.par;
  CompC C;
  comp_setup<double>(t, bn, S, C);
  const Kin k = kin_setup(t);
  const float jx = (float)(pj - c0 - C.ix), iy = (float)(pi - c0 - C.iy);
  const float inv = 1.0f / (float)(S * S * Sv);
  const float rt2 = k.rt * k.rt;
  float *dst = out + d.pad * (int64_t)Mc * 11 + p;
  const bool no_ie = mask && (mask[s] & kMaskModelIe);   // the Ie block comes from the kept model
  // spectral sub-sample offsets, once per thread (static register indices)
  float ov[GF_MAX_OVERSAMPLE];
#pragma unroll
  for (int tv = 0; tv < GF_MAX_OVERSAMPLE; ++tv) ov[tv] = tv < Sv ? sv_off(tv, Sv) : 0.0f;
  for (int pc0 = 0; pc0 < Mc; pc0 += kCubeCB) {
    float acc[11][kCubeCB];
#pragma unroll
    for (int j = 0; j < 11; ++j)
#pragma unroll
      for (int c = 0; c < kCubeCB; ++c) acc[j][c] = 0.0f;
    // sub-sample offsets formed as in comp_setup (the same values as C.ox,
    // C.oy, without indexing those arrays in a rolled loop)
    const float twoS = 2.0f * (float)S;
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      const float dy = iy + fmaf(-twoS, C.fy, (float)(2 * b + 1 - S)) / twoS;
#pragma unroll 1
      for (int a = 0; a < S; ++a) {
        const float dx = jx + fmaf(-twoS, C.fx, (float)(2 * a + 1 - S)) / twoS;
        const float xp = fmaf(dx, C.cs, dy * C.sn);
        const float yp = fmaf(-dx, C.sn, dy * C.cs);
        const float yi = C.iq2 * yp;
        const float r2 = fmaf(yi, yp, xp * xp);
        const bool nz = r2 > 0.0f;
        const float lt = fmaf(fast_log2(r2), C.a1, C.a0);     // log2 t
        const float tt = fast_exp2(lt);
        const float omt = 1.0f - tt;
        const float J = fast_exp2(C.b1 * omt);                 // I / Ie
        const float I = J * C.ie;
        const float IE = I * (C.bn * tt);
        const float wh = nz ? (IE * C.inv_n) * __builtin_amdgcn_rcpf(r2) : 0.0f;   // -(dI/dR)/R
        // R dR/dtheta
        const float rx = fmaf(-xp, C.cs, yi * C.sn);
        const float ry = fmaf(-xp, C.sn, -yi * C.cs);
        const float rphi = xp * yp * (1.0f - C.iq2);
        const float rq = -yi * yp * C.inv_q;
        const float R = sqrtf(r2);
        const float f = f_of_r(R, k);
        const float gr = g_of_r(R, k);
        const float V = fmaf(k.kv * xp, f, k.v0);
        const float kxg = k.kv * xp * gr;
        // coefficients of G (a) and of G (v - V)/sigma^2 (b)
        const float a0 = -wh * rx, a1 = -wh * ry, a2 = J, a3 = IE * (C.inv_n * C.inv_re);
        const float a4 = fmaf(I, C.dbn * omt, IE * (nz ? lt : 0.0f) * (0.69314718055994531f * C.inv_n));
        const float a5 = -wh * rq, a6 = -wh * rphi;
        const float b0 = I * fmaf(k.kv * f, -C.cs, kxg * rx);
        const float b1 = I * fmaf(k.kv * f, -C.sn, kxg * ry);
        const float b5 = I * kxg * rq;
        const float b6 = I * fmaf(k.kv * f, yp, kxg * rphi);
        const float b8 = I * (kTwoOverPi * xp * f);
        const float b9 = -I * k.kv * xp / (rt2 + r2);
        const float b10 = I * k.isg;
#pragma unroll
        for (int c = 0; c < kCubeCB; ++c) {
          const float vb = (float)(pc0 + c - cl) - V;
#pragma unroll
          for (int tv = 0; tv < GF_MAX_OVERSAMPLE; ++tv) {
            if (tv >= Sv) break;
            const float u = vb + ov[tv];
            const float e = fast_exp2(k.kg * u * u);
            const float h = e * u * k.is2;
            acc[0][c] = fmaf(a0, e, fmaf(b0, h, acc[0][c]));
            acc[1][c] = fmaf(a1, e, fmaf(b1, h, acc[1][c]));
            acc[2][c] = fmaf(a2, e, acc[2][c]);
            acc[3][c] = fmaf(a3, e, acc[3][c]);
            acc[4][c] = fmaf(a4, e, acc[4][c]);
            acc[5][c] = fmaf(a5, e, fmaf(b5, h, acc[5][c]));
            acc[6][c] = fmaf(a6, e, fmaf(b6, h, acc[6][c]));
            acc[7][c] = fmaf(I, h, acc[7][c]);
            acc[8][c] = fmaf(b8, h, acc[8][c]);
            acc[9][c] = fmaf(b9, h, acc[9][c]);
            acc[10][c] = fmaf(b10 * u, h, acc[10][c]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kCubeCB; ++c) {
      const int pc = pc0 + c;
      if (pc < Mc) {
#pragma unroll
        for (int j = 0; j < 11; ++j)
          if (!(j == 2 && no_ie)) dst[((int64_t)j * Mc + pc) * np] = acc[j][c] * inv;
      }
    }
  }
}

// Spectral valid convolution of nk padded cubes per cube (blockIdx.y = j):
// out[pad * Nc * nk + (j * Nc + c) * Mh*Mw + p] =
//   sum_u lsf[u] in[pad * Mc * nk + (j * Mc + c + Kl - 1 - u) * Mh*Mw + p],
// which is the channel layout of the spatial convolution's padded input.
__global__ __launch_bounds__(kThreads) void k_cube_lsf(const CubeDesc *__restrict__ desc, const Work *__restrict__ work,
                                                       const float *__restrict__ lsf_all, int Nc, int Kl, int nk,
                                                       const int *__restrict__ mask, const float *__restrict__ in,
                                                       float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const CubeDesc d = desc[s];
  const int np = d.Mh * d.Mw;
  const int p = w.unit * kThreads + (int)threadIdx.x;
  if (p >= np) return;
  const int j = blockIdx.y;
  if (nk > 1 && mask && (mask[s] & kMaskModelIe) && j == 2) return;   // the Ie block comes from the kept model
  const int Mc = Nc + Kl - 1;
  const float *src = in + d.pad * (int64_t)Mc * nk + (int64_t)j * Mc * np + p;
  float *dst = out + d.pad * (int64_t)Nc * nk + (int64_t)j * Nc * np + p;
  const float *l = lsf_all + d.lsf;
  for (int c = 0; c < Nc; ++c) {
    float acc = 0.0f;
    for (int u = 0; u < Kl; ++u) acc = fmaf(l[u], src[(int64_t)(c + Kl - 1 - u) * np], acc);
    dst[(int64_t)c * np] = acc;
  }
}

// The same for an LSF of KL taps known at compile time: each thread keeps a
// ring of the last KL input channels in registers, so every input value is
// loaded once (the generic kernel loads it KL times); the sums run over u in
// the same order, so both give the same bits.
template <int KL>
__global__ __launch_bounds__(kThreads) void k_cube_lsf_t(const CubeDesc *__restrict__ desc,
                                                         const Work *__restrict__ work,
                                                         const float *__restrict__ lsf_all, int Nc, int nk,
                                                         const int *__restrict__ mask, const float *__restrict__ in,
                                                         float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const int s = w.stamp;
  if (mask && !mask[s]) return;
  const CubeDesc d = desc[s];
  const int np = d.Mh * d.Mw;
  const int p = w.unit * kThreads + (int)threadIdx.x;
  if (p >= np) return;
  const int j = blockIdx.y;
  if (nk > 1 && mask && (mask[s] & kMaskModelIe) && j == 2) return;   // the Ie block comes from the kept model
  const int Mc = Nc + KL - 1;
  const float *src = in + d.pad * (int64_t)Mc * nk + (int64_t)j * Mc * np + p;
  float *dst = out + d.pad * (int64_t)Nc * nk + (int64_t)j * Nc * np + p;
  float lw[KL], win[KL];
#pragma unroll
  for (int u = 0; u < KL; ++u) lw[u] = lsf_all[d.lsf + u];
  // win[(i) % KL] holds input channel i once it is loaded
#pragma unroll
  for (int i = 0; i < KL - 1; ++i) win[i] = src[(int64_t)i * np];
  for (int c0 = 0; c0 < Nc; c0 += KL) {
#pragma unroll
    for (int r = 0; r < KL; ++r) {
      const int c = c0 + r;
      if (c >= Nc) break;
      // newest input: channel c + KL - 1, slot (r + KL - 1) % KL since c0 % KL == 0
      win[(r + KL - 1) % KL] = src[(int64_t)(c + KL - 1) * np];
      float acc = 0.0f;
#pragma unroll
      for (int u = 0; u < KL; ++u) acc = fmaf(lw[u], win[(r + KL - 1 - u) % KL], acc);
      dst[(int64_t)c * np] = acc;
    }
  }
}

// out[v] += continuum over every voxel of each cube (flat stamps).
__global__ __launch_bounds__(kThreads) void k_cube_cont(const StampDesc *__restrict__ desc, const Work *__restrict__ work,
                                                        const double *__restrict__ theta, float *__restrict__ m) {
  const Work w = work[blockIdx.x];
  const StampDesc d = desc[w.stamp];
  const int npix = d.H * d.W;
  const float cont = (float)theta[d.par + kNPC];
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = w.unit * kPixChunk + k * kThreads + (int)threadIdx.x;
    if (p < npix) m[d.pix + p] += cont;
  }
}

// Jacobian cubes in parameter order: out[12 pix + q * nvox + v] from the 11
// convolved derivative channels jc[11 pix + j * nvox + v] (j = q below the
// continuum, q - 1 above it) and ones for the continuum.
__global__ __launch_bounds__(kThreads) void k_cube_jac_assemble(const StampDesc *__restrict__ desc,
                                                                const Work *__restrict__ work,
                                                                const float *__restrict__ jc, float *__restrict__ out) {
  const Work w = work[blockIdx.x];
  const StampDesc d = desc[w.stamp];
  const int npix = d.H * d.W;
  for (int k = 0; k < kPixChunk / kThreads; ++k) {
    const int p = w.unit * kPixChunk + k * kThreads + (int)threadIdx.x;
    if (p >= npix) break;
    for (int q = 0; q < GF_CUBE_NPAR; ++q) {
      const float v = q == kNPC ? 1.0f : jc[d.pix * (int64_t)11 + (int64_t)(q < kNPC ? q : q - 1) * npix + p];
      out[d.pix * (int64_t)GF_CUBE_NPAR + (int64_t)q * npix + p] = v;
    }
  }
}

// theta = clip(start, lo, hi) element-wise (n values).
__global__ void k_cube_clip(int64_t n, const double *__restrict__ start, const double *__restrict__ lo,
                            const double *__restrict__ hi, double *__restrict__ theta) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = start[i];
  if (lo) v = fmax(v, lo[i]);
  if (hi) v = fmin(v, hi[i]);
  theta[i] = v;
}

// ------------------------------------------------------------ launchers

#define GF_CUBE_S(MACRO) \
  switch (S) {           \
    case 1: MACRO(1); break; \
    case 2: MACRO(2); break; \
    case 3: MACRO(3); break; \
    case 4: MACRO(4); break; \
    case 5: MACRO(5); break; \
    case 6: MACRO(6); break; \
    case 7: MACRO(7); break; \
    case 8: MACRO(8); break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_cube_eval(hipStream_t st, const CubeDesc *desc, const Work *work, int n_work, const double *theta,
                            const float4 *bn, int Nc, int Kl, int S, int Sv, const int *mask, float *out) {
  if (n_work == 0) return hipSuccess;
  ProfScope ps(st, "k_cube_eval");
#define GF_CE(SS) hipLaunchKernelGGL((k_cube_eval<SS>), dim3((unsigned)n_work), dim3(kThreads), 0, st, desc, work, \
                                     theta, bn, Nc, Kl, Sv, mask, out)
  GF_CUBE_S(GF_CE)
#undef GF_CE
  return hipGetLastError();
}

hipError_t launch_cube_jac(hipStream_t st, const CubeDesc *desc, const Work *work, int n_work, const double *theta,
                           const float4 *bn, int Nc, int Kl, int S, int Sv, const int *mask, float *out) {
  if (n_work == 0) return hipSuccess;
  ProfScope ps(st, "k_cube_jac");
#define GF_CJ(SS) hipLaunchKernelGGL((k_cube_jac<SS>), dim3((unsigned)n_work), dim3(kThreads), 0, st, desc, work, \
                                     theta, bn, Nc, Kl, Sv, mask, out)
  GF_CUBE_S(GF_CJ)
#undef GF_CJ
  return hipGetLastError();
}

hipError_t launch_cube_lsf(hipStream_t st, const CubeDesc *desc, const Work *work, int n_work, const float *lsf,
                           int Nc, int Kl, int nk, const int *mask, const float *in, float *out) {
  if (n_work == 0) return hipSuccess;
  ProfScope ps(st, "k_cube_lsf");
  const dim3 grid((unsigned)n_work, (unsigned)nk);
#define GF_CL(KK)                                                                                                  \
  case KK:                                                                                                         \
    hipLaunchKernelGGL((k_cube_lsf_t<KK>), grid, dim3(kThreads), 0, st, desc, work, lsf, Nc, nk, mask, in, out); \
    break;
  switch (Kl) {
    GF_CL(1) GF_CL(3) GF_CL(5) GF_CL(7) GF_CL(9) GF_CL(11) GF_CL(13) GF_CL(15)
    default:
      hipLaunchKernelGGL(k_cube_lsf, grid, dim3(kThreads), 0, st, desc, work, lsf, Nc, Kl, nk, mask, in, out);
  }
#undef GF_CL
  return hipGetLastError();
}

hipError_t launch_cube_cont(hipStream_t st, const gf_batch *flat, const double *theta, float *m) {
  dim3 grid((unsigned)flat->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cube_cont, grid, blk, 0, st, flat->d_desc, flat->d_pix, theta, m);
  return hipGetLastError();
}

hipError_t launch_cube_jac_assemble(hipStream_t st, const gf_batch *flat, const float *jc, float *out) {
  dim3 grid((unsigned)flat->h_pix.size()), blk(kThreads);
  if (grid.x == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cube_jac_assemble, grid, blk, 0, st, flat->d_desc, flat->d_pix, jc, out);
  return hipGetLastError();
}

hipError_t launch_cube_clip(hipStream_t st, int64_t n, const double *start, const double *lo, const double *hi,
                            double *theta) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cube_clip, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, start, lo, hi, theta);
  return hipGetLastError();
}

}  // namespace gf

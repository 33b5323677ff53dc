// comp.h -- per-component constants of the Sersic evaluation (device code):
// centre split into integer and fractional parts, sub-sample offsets,
// rotation, axis ratio, and the exponents of the profile
//   I(R) = Ie exp(-b_n [(R/Re)^(1/n) - 1]),
// evaluated as exp2(log2 Ie + b_n log2(e) (1 - t)) with
// t = exp2(log2(R^2)/(2n) - log2(Re)/n).  Shared by the evaluation kernels
// and the LM kernels that form trial points.
#pragma once
#include "gf_internal.h"

namespace gf {

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Cubic Hermite lookup of b_n (from node values and slopes) and of db_n/dn
// (from node slopes and curvatures) in the FP32 table built on the host.
__device__ __forceinline__ void bn_lookup(float n, const float4 *__restrict__ tab, float &b, float &db) {
  const float h = (float)((kBnHi - kBnLo) / (kBnNodes - 1));
  float u = (n - (float)kBnLo) / h;
  u = fminf(fmaxf(u, 0.0f), (float)(kBnNodes - 1) - 1e-3f);
  const int i = (int)u;
  const float t = u - (float)i;
  const float4 p0 = tab[i], p1 = tab[i + 1];
  const float t2 = t * t, t3 = t2 * t;
  const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t, h01 = -2.f * t3 + 3.f * t2, h11 = t3 - t2;
  b = h00 * p0.x + h01 * p1.x + h * (h10 * p0.y + h11 * p1.y);
  db = h00 * p0.y + h01 * p1.y + h * (h10 * p0.z + h11 * p1.z);
}

// Per-component constants from the parameter vector (float or double).
// The sub-sample offsets relative to the fractional centre,
//   (s + 1/2)/S - 1/2 - f = ((2s + 1 - S) - 2S f) / (2S),
// take one FMA (exact numerator up to one rounding) and one division, so a
// sub-sample within 1e-7 px of the centre keeps its distance to full
// relative precision; the Sersic cusp makes the value at such a point very
// sensitive to that distance for large n.
template <typename TT>
__device__ inline void comp_setup(const TT *__restrict__ t, const float4 *__restrict__ bn_tab, int S, CompC &c) {
  TT x0 = t[0], y0 = t[1];
  TT rx = rint(x0), ry = rint(y0);
  c.ix = (int)rx;
  c.iy = (int)ry;
  c.fx = (float)(x0 - rx);
  c.fy = (float)(y0 - ry);
  const float twoS = 2.0f * (float)S;
  for (int a = 0; a < S; ++a) {
    const float num = (float)(2 * a + 1 - S);
    c.ox[a] = fmaf(-twoS, c.fx, num) / twoS;
    c.oy[a] = fmaf(-twoS, c.fy, num) / twoS;
  }
  float ie = (float)t[2], re = (float)t[3], n = (float)t[4], q = (float)t[5], phi = (float)t[6];
  float sn, cs;
  sincosf(phi, &sn, &cs);
  float bn, dbn;
  bn_lookup(n, bn_tab, bn, dbn);
  c.cs = cs;
  c.sn = sn;
  c.cq = cs / q;
  c.sq = sn / q;
  c.iq2 = 1.0f / (q * q);
  c.a1 = 0.5f / n;
  c.a0 = -log2f(re) / n;
  c.b1 = bn * 1.4426950408889634f;
  c.lie = log2f(ie);
  c.ie = ie;
  c.re = re;
  c.n = n;
  c.q = q;
  c.bn = bn;
  c.dbn = dbn;
  c.inv_n = 1.0f / n;
  c.inv_re = 1.0f / re;
  c.inv_q = 1.0f / q;
}

}  // namespace gf

// bn_table.cpp -- host FP64 construction of the b_n table used by the
// evaluation kernels.
//
// b_n is defined by P(2n, b_n) = 1/2 (the radius Re holds half of the light),
// with P(a, x) = gamma(a, x)/Gamma(a).  The median of a gamma distribution
// lies below its mean, so b_n < 2n and the power series
//     P(a, x) = x^a e^-x / Gamma(a+1) * sum_{k>=0} x^k / ((a+1)(a+2)...(a+k))
// converges for every x we need.  The root is found by the Illinois variant
// of regula falsi on [0, 2n].  The first and second derivatives at each node
// come from fourth-order central differences of the FP64 node values (two
// guard nodes at each end), so the device can interpolate b_n from (b, b')
// and b'_n from (b', b'') with cubic Hermite polynomials, never differencing
// FP32 values.
#include <cmath>
#include <vector>

#include "gf_internal.h"

namespace gf {

static double gammp_series(double a, double x) {
  if (x <= 0.0) return 0.0;
  double term = 1.0, sum = 1.0, den = a;
  for (int k = 1; k < 20000; ++k) {
    den += 1.0;
    term *= x / den;
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return std::exp(a * std::log(x) - x - std::lgamma(a + 1.0)) * sum;
}

static double bn_root(double n) {
  const double a = 2.0 * n;
  double lo = 0.0, hi = a;
  double flo = -0.5, fhi = gammp_series(a, hi) - 0.5;
  int side = 0;
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 500; ++it) {
    x = (lo * fhi - hi * flo) / (fhi - flo);
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    const double fx = gammp_series(a, x) - 0.5;
    if (fx == 0.0) break;
    if ((fx > 0.0) == (fhi > 0.0)) {
      hi = x;
      fhi = fx;
      if (side == 1) flo *= 0.5;
      side = 1;
    } else {
      lo = x;
      flo = fx;
      if (side == -1) fhi *= 0.5;
      side = -1;
    }
    if (hi - lo < 4e-16 * x) break;
  }
  return x;
}

std::vector<float4> build_bn_table() {
  const double h = (kBnHi - kBnLo) / (kBnNodes - 1);
  std::vector<double> b(kBnNodes + 4);
  for (int i = -2; i < kBnNodes + 2; ++i) b[i + 2] = bn_root(kBnLo + i * h);
  std::vector<float4> tab(kBnNodes);
  for (int i = 0; i < kBnNodes; ++i) {
    const double *c = &b[i + 2];
    const double d1 = (-c[2] + 8.0 * c[1] - 8.0 * c[-1] + c[-2]) / (12.0 * h);
    const double d2 = (-c[2] + 16.0 * c[1] - 30.0 * c[0] + 16.0 * c[-1] - c[-2]) / (12.0 * h * h);
    tab[i] = make_float4((float)c[0], (float)d1, (float)d2, 0.0f);
  }
  return tab;
}

}  // namespace gf

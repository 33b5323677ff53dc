// fft_dft.h -- complex helpers and the in-register DFT butterflies shared by
// the FFT convolution kernels: radices 2, 3, 4, 5 and 8 directly, the
// composites 6 ... 32 by one Cooley-Tukey split with compile-time twiddles.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace gf {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }   // i a
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i a


// ------------------------------------------------------------ small DFTs
// Forward: X_k = sum_n x_n exp(-2 pi i n k / R); inverse uses +i.
template <bool INV>
__device__ __forceinline__ void dft2(float2 *v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2 *v) {
  const float s3 = 0.86602540378443865f;
  float2 a = v[0], b = v[1], c = v[2];
  float2 t1 = cadd(b, c);
  float2 t2 = make_float2(fmaf(-0.5f, t1.x, a.x), fmaf(-0.5f, t1.y, a.y));
  float2 m = mul_i(cscale(csub(b, c), s3));
  v[0] = cadd(a, t1);
  v[1] = INV ? cadd(t2, m) : csub(t2, m);
  v[2] = INV ? csub(t2, m) : cadd(t2, m);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 *v) {
  float2 a = v[0], b = v[1], c = v[2], d = v[3];
  float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
  float2 m = mul_i(d1);
  v[0] = cadd(s0, s1);
  v[2] = csub(s0, s1);
  v[1] = INV ? cadd(d0, m) : csub(d0, m);
  v[3] = INV ? csub(d0, m) : cadd(d0, m);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2 *v) {
  const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
  const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
  float2 a = v[0];
  float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  float2 p1 = make_float2(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
  float2 p2 = make_float2(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
  float2 q1 = mul_i(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  float2 q2 = mul_i(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v[0] = make_float2(a.x + t1.x + t2.x, a.y + t1.y + t2.y);
  v[1] = INV ? cadd(p1, q1) : csub(p1, q1);
  v[4] = INV ? csub(p1, q1) : cadd(p1, q1);
  v[2] = INV ? cadd(p2, q2) : csub(p2, q2);
  v[3] = INV ? csub(p2, q2) : cadd(p2, q2);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2 *v) {
  const float r = 0.70710678118654752f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // o[k] *= w^k, w = exp(-+ i pi/4)
  float2 o1 = INV ? make_float2(r * (o[1].x - o[1].y), r * (o[1].x + o[1].y))
                  : make_float2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
  float2 o2 = INV ? mul_i(o[2]) : mul_mi(o[2]);
  float2 o3 = INV ? make_float2(-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y))
                  : make_float2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// ------------------------------------------------------------ composite DFTs
// Twiddles W_R^M = exp(-2 pi i M / R) of the in-register composite DFTs are
// compile-time constants: cos and sin of 2 pi M / R evaluated in double by
// octant reduction and Taylor series (|x| <= pi/4, 14 terms), then rounded.
constexpr double kPiD = 3.14159265358979323846;
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// (cos, sin) of 2 pi m / r for integers m, r > 0.
struct CS {
  double c, s;
};
constexpr CS unit_root(int m, int r) {
  m %= r;
  if (m < 0) m += r;
  const int oct = (8 * m) / r;                                   // octant 0..7
  const double x = 2.0 * kPiD * ((double)m / r) - oct * (kPiD / 4.0);   // [0, pi/4)
  double c, s;
  if (oct % 2 == 0) {
    c = taylor_cos(x);
    s = taylor_sin(x);
  } else {
    const double y = kPiD / 4.0 - x;                             // phi = pi/2 - y
    c = taylor_sin(y);
    s = taylor_cos(y);
  }
  switch (oct / 2) {
    case 0: return CS{c, s};
    case 1: return CS{-s, c};
    case 2: return CS{-c, -s};
    default: return CS{s, -c};
  }
}

// a * W_R^M (forward) or a * conj(W_R^M) (inverse).
template <int R, int M, bool INV>
__device__ __forceinline__ float2 twc(float2 a) {
  if constexpr (M % R == 0) {
    return a;
  } else {
    constexpr CS w = unit_root(M, R);
    constexpr float c = (float)w.c, sn = (float)w.s;
    return INV ? make_float2(fmaf(a.x, c, -a.y * sn), fmaf(a.y, c, a.x * sn))
               : make_float2(fmaf(a.x, c, a.y * sn), fmaf(a.y, c, -a.x * sn));
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 *v);

// Slot B*n1 + n2 holds Y[n2][k1 = n1] after the first stage; it is scaled
// by W_R^{n2 k1}.
template <int A, int B, bool INV, int... I>
__device__ __forceinline__ void tw_apply(float2 *v, std::integer_sequence<int, I...>) {
  ((v[I] = twc<A * B, (I / B) * (I % B), INV>(v[I])), ...);
}

// Length R = A B by one Cooley-Tukey split, in place, natural order in and
// out: n = B n1 + n2, k = k1 + A k2,
//   X[k1 + A k2] = sum_n2 W_B^{n2 k2} W_R^{n2 k1} sum_n1 x[B n1 + n2] W_A^{n1 k1}.
template <int A, int B, bool INV>
__device__ __forceinline__ void dft_ab(float2 *v) {
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    float2 t[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
    dft<A, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) v[B * k1 + n2] = t[k1];
  }
  tw_apply<A, B, INV>(v, std::make_integer_sequence<int, A * B>{});
  float2 o[A * B];
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    float2 t[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) t[n2] = v[B * k1 + n2];
    dft<B, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) o[k1 + A * k2] = t[k2];
  }
#pragma unroll
  for (int i = 0; i < A * B; ++i) v[i] = o[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 *v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 5) dft5<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 6) dft_ab<2, 3, INV>(v);
  else if constexpr (R == 9) dft_ab<3, 3, INV>(v);
  else if constexpr (R == 10) dft_ab<2, 5, INV>(v);
  else if constexpr (R == 12) dft_ab<4, 3, INV>(v);
  else if constexpr (R == 15) dft_ab<3, 5, INV>(v);
  else if constexpr (R == 16) dft_ab<4, 4, INV>(v);
  else if constexpr (R == 18) dft_ab<2, 9, INV>(v);
  else if constexpr (R == 20) dft_ab<4, 5, INV>(v);
  else if constexpr (R == 24) dft_ab<8, 3, INV>(v);
  else if constexpr (R == 25) dft_ab<5, 5, INV>(v);
  else if constexpr (R == 27) dft_ab<3, 9, INV>(v);
  else if constexpr (R == 32) dft_ab<8, 4, INV>(v);
  else static_assert(R == 2, "unsupported radix");
}

}  // namespace gf

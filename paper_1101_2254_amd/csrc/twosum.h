// twosum.h -- FP32 (hi, lo) pairs updated by error-free TwoSum (Knuth) and
// their wave64 shuffle sum, shared by the reduction kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

struct F2 {
  float hi, lo;
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  F2 r;
  r.hi = s + e;
  r.lo = e - (r.hi - s);
  return r;
}

__device__ __forceinline__ F2 f2_add1(F2 a, float v) {
  float s, e;
  two_sum(a.hi, v, s, e);
  F2 r;
  r.hi = s;
  r.lo = a.lo + e;
  return r;
}

__device__ __forceinline__ F2 wave_sum(F2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    F2 o;
    o.hi = __shfl_xor(v.hi, off, 64);
    o.lo = __shfl_xor(v.lo, off, 64);
    v = f2_add(v, o);
  }
  return v;
}

}  // namespace gf

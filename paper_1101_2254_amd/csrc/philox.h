// philox.h -- Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC 2011) as
// device functions, shared by the random-number and sampler kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gf {

struct U256 {
  uint64_t w[4];
};

__device__ __forceinline__ U256 ctr_add(const U256 &c, uint64_t b) {
  U256 r = c;
  r.w[0] = c.w[0] + b;
  uint64_t carry = r.w[0] < b ? 1u : 0u;
  for (int i = 1; i < 4; ++i) {
    r.w[i] = c.w[i] + carry;
    carry = (carry && r.w[i] == 0) ? 1u : 0u;
  }
  return r;
}

// Ten rounds; the key advances by the two Weyl increments between rounds.
__device__ __forceinline__ void philox10(U256 &c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c.w[0], hi0 = __umul64hi(M0, c.w[0]);
    const uint64_t lo1 = M1 * c.w[2], hi1 = __umul64hi(M1, c.w[2]);
    const uint64_t n0 = hi1 ^ c.w[1] ^ k0, n2 = hi0 ^ c.w[3] ^ k1;
    c.w[0] = n0;
    c.w[1] = lo1;
    c.w[2] = n2;
    c.w[3] = lo0;
  }
}

// Uniform in (0, 1) from the top 24 bits of a word (exact in FP64).
__device__ __forceinline__ double u24(uint64_t w) { return ((double)(w >> 40) + 0.5) * 0x1p-24; }

inline U256 to_u256(const uint64_t *c) {
  U256 r;
  for (int i = 0; i < 4; ++i) r.w[i] = c ? c[i] : 0;
  return r;
}

}  // namespace gf

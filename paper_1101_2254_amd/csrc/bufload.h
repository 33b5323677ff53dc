// bufload.h -- range-checked loads through buffer resources.  A raw buffer
// load whose byte offset lies past the resource's size returns zero without
// touching memory, so a batch of loads with some out-of-range elements can be
// issued unconditionally (no branch, hence no wait inside a branch) and the
// zeros come for free.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gf {

typedef int i32x2_t __attribute__((ext_vector_type(2)));

// Resource over [p, p + bytes); bytes < 2^31.  Third dword: raw 32-bit
// accesses on the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

constexpr uint32_t kOutOfRange = 0x80000000u;   // any byte offset past every resource

__device__ __forceinline__ float bload_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__device__ __forceinline__ float2 bload_f32x2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const i32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return make_float2(__int_as_float(v[0]), __int_as_float(v[1]));
}

}  // namespace gf

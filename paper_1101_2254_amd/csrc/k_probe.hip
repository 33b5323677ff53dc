// k_probe.hip -- roofline calibration probes: the achievable HBM bandwidth
// (a streaming triad), the FP32 FMA issue rate and the rate of the hardware
// log2/exp2 instructions on the device the library runs on.  They give the
// denominators the kernels' roofline fractions can also be read against.
#include "gf_internal.h"

namespace gf {

__global__ __launch_bounds__(256) void k_probe_triad(const float4 *__restrict__ a, const float4 *__restrict__ b,
                                                     float4 *__restrict__ c, int64_t n4, float s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 x = a[i], y = b[i];
    c[i] = make_float4(fmaf(s, y.x, x.x), fmaf(s, y.y, x.y), fmaf(s, y.z, x.z), fmaf(s, y.w, x.w));
  }
}

// Eight independent FMA chains per thread.
__global__ __launch_bounds__(256) void k_probe_fma(int iters, float a, float *__restrict__ out) {
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (float)(threadIdx.x + j) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = fmaf(v[j], a, 0.5f);
  }
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) t += v[j];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// Four independent chains of exp2(log2(x) * a) per thread (two transcendentals per step).
__global__ __launch_bounds__(256) void k_probe_trans(int iters, float a, float *__restrict__ out) {
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = 1.0f + (float)(threadIdx.x + j) * 1e-4f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(v[j]) * a);
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = v[0] + v[1] + v[2] + v[3];
}

}  // namespace gf

using namespace gf;

extern "C" gf_status gf_probe(gf_ctx *c, int kind, int64_t n, int reps, double *result) {
  if (!c || !result || reps <= 0 || n <= 0) {
    if (c) c->err = "gf_probe: bad argument";
    return GF_EINVAL;
  }
  hipStream_t st = c->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    c->err = "gf_probe: event creation failed";
    return GF_EDEVICE;
  }
  int dev_cus = 0;
  (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device);
  gf_status rc = GF_OK;
  float *buf = nullptr;
  const int blocks = std::max(1, dev_cus) * 64;
  if (kind == 0) {
    const int64_t n4 = (n + 3) / 4;
    if (hipMalloc((void **)&buf, (size_t)n4 * 3 * sizeof(float4)) != hipSuccess) {
      c->err = "gf_probe: allocation failed";
      rc = GF_ENOMEM;
    } else {
      (void)hipMemsetAsync(buf, 0, (size_t)n4 * 3 * sizeof(float4), st);
      const float4 *a = (const float4 *)buf, *b = a + n4;
      float4 *o = (float4 *)buf + 2 * n4;
      hipLaunchKernelGGL(k_probe_triad, dim3(blocks * 4), dim3(256), 0, st, a, b, o, n4, 1.5f);
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_probe_triad, dim3(blocks * 4), dim3(256), 0, st, a, b, o, n4, 1.5f);
      (void)hipEventRecord(e1, st);
    }
  } else if (kind == 1 || kind == 2) {
    if (hipMalloc((void **)&buf, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) {
      c->err = "gf_probe: allocation failed";
      rc = GF_ENOMEM;
    } else {
      const int iters = (int)std::min<int64_t>(n, 1 << 24);
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r) {
        if (kind == 1)
          hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, iters, 0.999f, buf);
        else
          hipLaunchKernelGGL(k_probe_trans, dim3(blocks), dim3(256), 0, st, iters, 0.999f, buf);
      }
      (void)hipEventRecord(e1, st);
    }
  } else {
    c->err = "gf_probe: unknown kind";
    rc = GF_EINVAL;
  }
  if (rc == GF_OK) {
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      c->err = "gf_probe: timing failed";
      rc = GF_EDEVICE;
    } else {
      const double s = ms * 1e-3;
      const double threads = (double)blocks * 256;
      const double iters = (double)std::min<int64_t>(n, 1 << 24);
      if (kind == 0) *result = (double)((n + 3) / 4) * 16.0 * 3.0 * reps / s / 1e9;         // GB/s
      else if (kind == 1) *result = threads * iters * 8.0 * 2.0 * reps / s / 1e12;        // TFLOP/s
      else *result = threads * iters * 4.0 * 2.0 * reps / s / 1e9;                        // G transcendental ops/s
    }
  }
  if (buf) (void)hipFree(buf);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

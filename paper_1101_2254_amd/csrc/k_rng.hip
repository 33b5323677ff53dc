// k_rng.hip -- on-device counter-based random numbers for the training and
// evaluation stamps of the learned proposal: Philox4x64-10 (Salmon, Moraes,
// Dror & Shaw, SC 2011), Gaussian noise by the Box-Muller transform, and
// draws of single-Sersic parameters from the prior box of the uneven-batch
// workload (side N: n ~ U[0.5, 6], Re ~ U[2, N/4], q ~ U[0.2, 1],
// PA ~ U[0, pi], Ie log-uniform on [0.5, 5], centre N/2 + U[-1, 1] per axis,
// sky ~ U[0, 0.05]).
//
// Every value is a pure function of (key, counter): a block index b always
// uses counter base + b (256-bit addition), so results do not depend on the
// launch shape.
#include "gf_internal.h"
#include "philox.h"

namespace gf {

__global__ void k_philox_raw(uint64_t k0, uint64_t k1, U256 base, int64_t nblocks, uint64_t *__restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  U256 c = ctr_add(base, (uint64_t)b);
  philox10(c, k0, k1);
  for (int i = 0; i < 4; ++i) out[4 * b + i] = c.w[i];
}

// out[j] = clean[j] (0 if null) + sigma * z_j; block b gives z_{4b..4b+3}.
__global__ void k_normal_noise(uint64_t k0, uint64_t k1, U256 base, int64_t n, float sigma,
                               const float *__restrict__ clean, float *__restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j0 = 4 * b;
  if (j0 >= n) return;
  U256 c = ctr_add(base, (uint64_t)b);
  philox10(c, k0, k1);
  const double r1 = sqrt(-2.0 * log(u24(c.w[0]))), r2 = sqrt(-2.0 * log(u24(c.w[2])));
  double s1, c1, s2, c2;
  sincospi(2.0 * u24(c.w[1]), &s1, &c1);
  sincospi(2.0 * u24(c.w[3]), &s2, &c2);
  const float z[4] = {(float)(r1 * c1), (float)(r1 * s1), (float)(r2 * c2), (float)(r2 * s2)};
  if (j0 + 4 <= n && ((reinterpret_cast<uintptr_t>(out + j0) | (clean ? reinterpret_cast<uintptr_t>(clean + j0) : 0)) & 15) == 0) {
    float4 v = clean ? *reinterpret_cast<const float4 *>(clean + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
    v.x = fmaf(sigma, z[0], v.x);
    v.y = fmaf(sigma, z[1], v.y);
    v.z = fmaf(sigma, z[2], v.z);
    v.w = fmaf(sigma, z[3], v.w);
    *reinterpret_cast<float4 *>(out + j0) = v;
  } else {
    for (int i = 0; i < 4 && j0 + i < n; ++i) out[j0 + i] = fmaf(sigma, z[i], clean ? clean[j0 + i] : 0.f);
  }
}

// Stamp i takes blocks base + 2i and base + 2i + 1 (eight uniforms u0..u7).
__global__ void k_draw_prior(uint64_t k0, uint64_t k1, U256 base, int n, int side, float *__restrict__ theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double u[8];
  for (int h = 0; h < 2; ++h) {
    U256 c = ctr_add(base, 2ull * (uint64_t)i + (uint64_t)h);
    philox10(c, k0, k1);
    for (int j = 0; j < 4; ++j) u[4 * h + j] = u24(c.w[j]);
  }
  const double half = 0.5 * side;
  float *t = theta + 8 * (int64_t)i;
  t[0] = (float)(half + 2.0 * u[5] - 1.0);               // x0
  t[1] = (float)(half + 2.0 * u[6] - 1.0);               // y0
  t[2] = (float)(0.5 * exp(u[4] * 2.302585092994046));   // Ie: 0.5 * 10^u
  t[3] = (float)(2.0 + (0.25 * side - 2.0) * u[1]);      // Re
  t[4] = (float)(0.5 + 5.5 * u[0]);                      // n
  t[5] = (float)(0.2 + 0.8 * u[2]);                      // q
  t[6] = (float)(3.141592653589793 * u[3]);              // phi
  t[7] = (float)(0.05 * u[7]);                           // sky
}

// out[i] = lim * (2 u_i - 1), u_i from word i of the stream (block i/4, word i%4).
__global__ void k_init_uniform(uint64_t k0, uint64_t k1, U256 base, int64_t n, float lim, float *__restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * b >= n) return;
  U256 c = ctr_add(base, (uint64_t)b);
  philox10(c, k0, k1);
  for (int i = 0; i < 4 && 4 * b + i < n; ++i) out[4 * b + i] = (float)((double)lim * (2.0 * u24(c.w[i]) - 1.0));
}

hipError_t launch_philox_raw(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t nblocks,
                             uint64_t *out) {
  if (nblocks <= 0) return hipSuccess;
  ProfScope ps(st, "k_philox_raw");
  hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0, st, k0, k1, to_u256(ctr),
                     nblocks, out);
  return hipGetLastError();
}

hipError_t launch_normal_noise(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t n, float sigma,
                               const float *clean, float *out) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + 3) / 4;
  ProfScope ps(st, "k_normal_noise");
  hipLaunchKernelGGL(k_normal_noise, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, k0, k1, to_u256(ctr), n,
                     sigma, clean, out);
  return hipGetLastError();
}

hipError_t launch_draw_prior(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int n, int side,
                             float *theta) {
  if (n <= 0) return hipSuccess;
  ProfScope ps(st, "k_draw_prior");
  hipLaunchKernelGGL(k_draw_prior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k0, k1, to_u256(ctr), n, side,
                     theta);
  return hipGetLastError();
}

hipError_t launch_init_uniform(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t n, float lim,
                               float *out) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + 3) / 4;
  hipLaunchKernelGGL(k_init_uniform, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, k0, k1, to_u256(ctr), n,
                     lim, out);
  return hipGetLastError();
}

}  // namespace gf

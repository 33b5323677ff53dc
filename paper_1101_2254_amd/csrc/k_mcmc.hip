// k_mcmc.hip -- random-walk Metropolis over a batch of chains, each chain one
// stamp of the batch (the paper's third routine family, Sec. 2: Bayesian
// sampling of the same likelihood; steps 1-3 are unchanged, step 4 proposes
// and accepts).  Target: exp(-chi^2 / 2) times a flat prior on the box
// [lo, hi]; proposal theta' = theta + scale * z, z ~ N(0, I).
//
// Random numbers: chain c at step t uses Philox4x64-10 blocks with counter
// (b, c, step0 + t, stream): blocks b = 0..3 give the normals z_{4b..4b+3}
// by Box-Muller on 24-bit uniforms (pairs (w0, w1) and (w2, w3)), block 4
// word 0 gives the acceptance uniform u; accept iff ln u < -(chi2' - chi2)/2.
#include "gf_internal.h"
#include "philox.h"
#include "twosum.h"

namespace gf {

__device__ __forceinline__ U256 mcmc_ctr(int b, int chain, int64_t step, uint64_t stream) {
  U256 c;
  c.w[0] = (uint64_t)b;
  c.w[1] = (uint64_t)chain;
  c.w[2] = (uint64_t)step;
  c.w[3] = stream;
  return c;
}

// One wave per chain: lane j < P draws z_j and writes theta'_j; the chain is
// evaluated only if theta' lies in the box.
__global__ __launch_bounds__(64) void k_mcmc_propose(const StampDesc *__restrict__ desc,
                                                     const double *__restrict__ theta,
                                                     const double *__restrict__ scale,
                                                     const double *__restrict__ lo, const double *__restrict__ hi,
                                                     uint64_t k0, uint64_t k1, uint64_t stream, int64_t step0,
                                                     const int64_t *__restrict__ tstep, double *__restrict__ theta_t,
                                                     int *__restrict__ mask) {
  __shared__ int inside;
  const int s = blockIdx.x, j = threadIdx.x;
  const StampDesc d = desc[s];
  const int P = kNPC * d.ncomp + 1;
  if (j == 0) inside = 1;
  __syncthreads();
  if (j < P) {
    U256 c = mcmc_ctr(j >> 2, s, step0 + *tstep, stream);
    philox10(c, k0, k1);
    const int q = j & 3, pr = q >> 1;
    const double r = sqrt(-2.0 * log(u24(c.w[2 * pr])));
    double sn, cs;
    sincospi(2.0 * u24(c.w[2 * pr + 1]), &sn, &cs);
    const double z = r * ((q & 1) ? sn : cs);
    const int64_t i = d.par + j;
    const double v = theta[i] + (scale ? scale[i] : 0.0) * z;
    theta_t[i] = v;
    if ((lo && v < lo[i]) || (hi && v > hi[i])) atomicAnd(&inside, 0);
  }
  __syncthreads();
  if (j == 0) mask[s] = inside;
}

// chi^2 of the start point from the finished (hi, lo) pairs.
__global__ void k_mcmc_init(int n, const float2 *__restrict__ pairs, double *__restrict__ chi2,
                            int64_t *__restrict__ tstep) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) chi2[s] = (double)pairs[s].x + (double)pairs[s].y;
  if (s == 0) *tstep = 0;
}

// One wave per chain: finish chi^2' from the workgroup partials (fixed
// order), draw u, accept or keep, store the state every `thin` steps.
__global__ __launch_bounds__(64) void k_mcmc_accept(const StampDesc *__restrict__ desc,
                                                    const int32_t *__restrict__ pix_first,
                                                    const float2 *__restrict__ part, const int *__restrict__ mask,
                                                    uint64_t k0, uint64_t k1, uint64_t stream, int64_t step0,
                                                    const int64_t *__restrict__ tstep, double *__restrict__ theta,
                                                    const double *__restrict__ theta_t, double *__restrict__ chi2,
                                                    int32_t *__restrict__ accepted, float *__restrict__ samples,
                                                    int64_t n_par, int thin) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const StampDesc d = desc[s];
  const int P = kNPC * d.ncomp + 1;
  const int64_t t = *tstep;
  bool acc = false;
  double c2 = 0.0;
  if (mask[s]) {
    F2 r = {0.f, 0.f};
    for (int u = pix_first[s] + lane; u < pix_first[s + 1]; u += 64) {
      const float2 v = part[u];
      F2 x = {v.x, v.y};
      r = f2_add(r, x);
    }
    r = wave_sum(r);
    c2 = (double)r.hi + (double)r.lo;
    U256 c = mcmc_ctr(4, s, step0 + t, stream);
    philox10(c, k0, k1);
    acc = log(u24(c.w[0])) < -0.5 * (c2 - chi2[s]);
  }
  double v = 0.0;
  if (lane < P) {
    v = theta[d.par + lane];
    if (acc) {
      v = theta_t[d.par + lane];
      theta[d.par + lane] = v;
    }
    if (samples && (t + 1) % thin == 0) samples[((t + 1) / thin - 1) * n_par + d.par + lane] = (float)v;
  }
  if (lane == 0 && acc) {
    chi2[s] = c2;
    if (accepted) accepted[s] += 1;
  }
}

__global__ void k_mcmc_tick(int64_t *__restrict__ tstep) { *tstep += 1; }

hipError_t launch_mcmc_propose(hipStream_t st, const gf_batch *b, const double *theta, const double *scale,
                               const double *lo, const double *hi, uint64_t k0, uint64_t k1, uint64_t stream,
                               int64_t step0, const int64_t *tstep, double *theta_t, int *mask) {
  ProfScope ps(st, "k_mcmc_propose");
  hipLaunchKernelGGL(k_mcmc_propose, dim3(b->n), dim3(64), 0, st, b->d_desc, theta, scale, lo, hi, k0, k1, stream,
                     step0, tstep, theta_t, mask);
  return hipGetLastError();
}

hipError_t launch_mcmc_init(hipStream_t st, int n, const float2 *pairs, double *chi2, int64_t *tstep) {
  hipLaunchKernelGGL(k_mcmc_init, dim3((n + 255) / 256), dim3(256), 0, st, n, pairs, chi2, tstep);
  return hipGetLastError();
}

hipError_t launch_mcmc_accept(hipStream_t st, const gf_batch *b, const int32_t *first, const float2 *part,
                              const int *mask, uint64_t k0,
                              uint64_t k1, uint64_t stream, int64_t step0, int64_t *tstep, double *theta,
                              const double *theta_t, double *chi2, int32_t *accepted, float *samples, int thin) {
  {
    ProfScope ps(st, "k_mcmc_accept");
    hipLaunchKernelGGL(k_mcmc_accept, dim3(b->n), dim3(64), 0, st, b->d_desc, first, part, mask, k0, k1,
                       stream, step0, tstep, theta, theta_t, chi2, accepted, samples, b->n_par, thin);
  }
  hipLaunchKernelGGL(k_mcmc_tick, dim3(1), dim3(1), 0, st, tstep);
  return hipGetLastError();
}

}  // namespace gf

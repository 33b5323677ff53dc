// k_moments.hip -- default starting point of a single-Sersic fit from image
// moments: sky from the median of the outer frame, centre and shape from
// ramp-weighted first and second moments, effective radius from the curve of
// growth, Ie from the total flux at n = 2.  One workgroup per stamp.
//
// Curve of growth: pixel p (elliptical radius r_p about the centre, weight
// v_p) contributes v_p clamp(r - r_p + 1/2, 0, 1) to C(r), i.e. its weight is
// spread evenly over a unit-width annulus; Re solves C(Re) = sum(v)/2.  C is
// continuous and piecewise linear in r and in every r_p and v_p, so Re does
// not jump when the order of nearly equal radii changes.
#include "gf_internal.h"

namespace gf {

constexpr int kMomThreads = 256;
constexpr int kMomBorder = 4;
constexpr int kMomBisect = 40;

__device__ double mom_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kMomThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ bool in_frame(int r, int c, int H, int W) {
  return r < kMomBorder || r >= H - kMomBorder || c < kMomBorder || c >= W - kMomBorder;
}

__global__ __launch_bounds__(kMomThreads) void k_moments(const StampDesc *__restrict__ desc,
                                                         const float *__restrict__ data, int p2,
                                                         double *__restrict__ theta) {
  extern __shared__ double mom_lds[];
  double *red = mom_lds;                                   // kMomThreads doubles
  float *fr = reinterpret_cast<float *>(mom_lds + kMomThreads);   // p2 floats
  __shared__ int cnt;
  const StampDesc d = desc[blockIdx.x];
  const int H = d.H, W = d.W, npx = H * W;
  const float *img = data + d.img;
  const int tid = threadIdx.x;
  // frame values, padded with +inf to a power of two, sorted (bitonic)
  if (tid == 0) cnt = 0;
  __syncthreads();
  for (int i = tid; i < npx; i += kMomThreads) {
    const int r = i / W, c = i - r * W;
    if (in_frame(r, c, H, W)) fr[atomicAdd(&cnt, 1)] = img[i];
  }
  __syncthreads();
  const int nf = cnt;
  for (int i = nf + tid; i < p2; i += kMomThreads) fr[i] = INFINITY;
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < p2; i += kMomThreads) {
        const int ij = i ^ j;
        if (ij > i) {
          const float a = fr[i], b = fr[ij];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            fr[i] = b;
            fr[ij] = a;
          }
        }
      }
      __syncthreads();
    }
  const double sky = (nf & 1) ? (double)fr[nf / 2] : 0.5 * ((double)fr[nf / 2 - 1] + (double)fr[nf / 2]);
  double q2 = 0.0;
  for (int i = tid; i < nf; i += kMomThreads) {
    const double e = fr[i] - sky;
    q2 += e * e;
  }
  const double rms = sqrt(mom_sum(q2, red) / nf);
  const double inv_s = rms > 0.0 ? 1.0 / rms : 0.0;
  // zeroth and first moments, total flux
  double s0 = 0.0, sx = 0.0, sy = 0.0, sf = 0.0;
  for (int i = tid; i < npx; i += kMomThreads) {
    const int r = i / W, c = i - r * W;
    const double e = img[i] - sky;
    const double v = e * fmin(fmax(e * inv_s - 2.0, 0.0), 1.0);
    s0 += v;
    sx += v * c;
    sy += v * r;
    sf += e;
  }
  s0 = mom_sum(s0, red);
  sx = mom_sum(sx, red);
  sy = mom_sum(sy, red);
  const double F = mom_sum(sf, red);
  double *th = theta + d.par;
  double xc = 0.5 * W, yc = 0.5 * H, q = 1.0, phi = 0.0, re = 2.0;
  if (s0 > 0.0) {
    xc = sx / s0;
    yc = sy / s0;
    double mxx = 0.0, myy = 0.0, mxy = 0.0;
    for (int i = tid; i < npx; i += kMomThreads) {
      const int r = i / W, c = i - r * W;
      const double e = img[i] - sky;
      const double v = e * fmin(fmax(e * inv_s - 2.0, 0.0), 1.0);
      const double dx = c - xc, dy = r - yc;
      mxx += v * dx * dx;
      myy += v * dy * dy;
      mxy += v * dx * dy;
    }
    mxx = mom_sum(mxx, red) / s0;
    myy = mom_sum(myy, red) / s0;
    mxy = mom_sum(mxy, red) / s0;
    const double hm = 0.5 * (mxx + myy), dm = sqrt(0.25 * (mxx - myy) * (mxx - myy) + mxy * mxy);
    const double l1 = hm + dm, l2 = fmax(hm - dm, 0.0);
    q = l1 > 0.0 ? fmin(1.0, fmax(0.05, sqrt(l2 / l1))) : 1.0;
    phi = 0.5 * atan2(2.0 * mxy, mxx - myy);
    if (phi < 0.0) phi += 3.141592653589793;
    const double cs = cos(phi), sn = sin(phi), iq = 1.0 / q;
    // bisection on C(r) = s0 / 2 over [0, rmax]
    const double rmax = (sqrt((double)H * H + (double)W * W) + 1.0) * iq + 1.0;
    const double half = 0.5 * s0;
    double lo = 0.0, hi = rmax, clo = 0.0, chi = s0;
    for (int it = 0; it < kMomBisect; ++it) {
      const double mid = 0.5 * (lo + hi);
      double cm = 0.0;
      for (int i = tid; i < npx; i += kMomThreads) {
        const int r = i / W, c = i - r * W;
        const double e = img[i] - sky;
        const double v = e * fmin(fmax(e * inv_s - 2.0, 0.0), 1.0);
        if (v == 0.0) continue;
        const double dx = c - xc, dy = r - yc;
        const double xp = dx * cs + dy * sn, yp = (dy * cs - dx * sn) * iq;
        const double rp = sqrt(xp * xp + yp * yp);
        cm += v * fmin(fmax(mid - rp + 0.5, 0.0), 1.0);
      }
      cm = mom_sum(cm, red);
      if (cm >= half) {
        hi = mid;
        chi = cm;
      } else {
        lo = mid;
        clo = cm;
      }
    }
    re = chi > clo ? lo + (hi - lo) * (half - clo) / (chi - clo) : 0.5 * (lo + hi);
    re = fmax(re, 0.1);
  }
  if (tid == 0) {
    // n = 2: b_2 is the root of P(4, b) = 1/2; Gamma(4) = 6
    const double b2 = 3.672060748850898;
    const double norm = 2.0 * 3.141592653589793 * 2.0 * re * re * q * exp(b2) * pow(b2, -4.0) * 6.0;
    th[0] = xc;
    th[1] = yc;
    th[2] = fmax(F / norm, 1e-3);
    th[3] = re;
    th[4] = 2.0;
    th[5] = q;
    th[6] = phi;
    th[7] = sky;
  }
}

size_t moments_lds_bytes(int p2) { return (size_t)kMomThreads * sizeof(double) + (size_t)p2 * sizeof(float); }

hipError_t launch_moments(hipStream_t st, const gf_batch *b, const float *data, int p2, double *theta) {
  ProfScope ps(st, "k_moments");
  hipLaunchKernelGGL(k_moments, dim3(b->n), dim3(kMomThreads), moments_lds_bytes(p2), st, b->d_desc, data, p2, theta);
  return hipGetLastError();
}

}  // namespace gf

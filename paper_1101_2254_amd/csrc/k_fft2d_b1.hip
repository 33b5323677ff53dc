// k_fft2d_b1.hip -- the one-workgroup FFT convolution kernels of bucket 1
// (side classes kF2dBucketEnd[1 - 1] .. kF2dBucketEnd[1] - 1; see fft2d_impl.h).
#include "fft2d_impl.h"

namespace gf {
hipError_t f2d_launch_b1(int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc, const PathDesc *path,
                         const float2 *tw_all, const Work *list, const float *in, float *out, const float2 *otf,
                         float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  return f2_launch_bucket<1>(mode, st, n, n_ch, desc, path, tw_all, list, in, out, otf, otf_out, mask, ep);
}
}  // namespace gf

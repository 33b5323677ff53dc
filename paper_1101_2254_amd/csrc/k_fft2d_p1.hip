// k_fft2d_p1.hip -- the one-workgroup FFT convolution kernels of side classes
// kF2dPart[1] .. kF2dPart[2] - 1 (see fft2d_impl.h).
#include "fft2d_impl.h"

namespace gf {
hipError_t f2d_launch_p1(int cls, int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc,
                         const PathDesc *path, const float2 *tw, const Work *list, const float *in, float *out,
                         const float2 *otf, float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  return f2_launch_part<kF2dPart[1], kF2dPart[2]>(cls, mode, st, n, n_ch, desc, path, tw, list, in, out, otf,
                                                        otf_out, mask, ep);
}
}  // namespace gf

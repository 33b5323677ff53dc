// k_fft2d_p3.hip -- the one-workgroup FFT convolution kernels of side classes
// kF2dPart[3] .. kF2dPart[4] - 1 (see fft2d_impl.h).
#include "fft2d_impl.h"

namespace gf {
hipError_t f2d_launch_p3(int cls, int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc,
                         const PathDesc *path, const float2 *tw, const Work *list, const float *in, float *out,
                         const float2 *otf, float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  return f2_launch_part<kF2dPart[3], kF2dPart[4]>(cls, mode, st, n, n_ch, desc, path, tw, list, in, out, otf,
                                                        otf_out, mask, ep);
}
}  // namespace gf

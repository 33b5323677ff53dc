// k_fft2d.hip -- host launchers of the one-workgroup FFT convolution
// (kernels in fft2d_impl.h, built by k_fft2d_p0 .. p3).
#include "fft2d_impl.h"

namespace gf {

static hipError_t f2d_launch(int cls, int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc,
                             const PathDesc *path, const float2 *tw, const Work *list, const float *in, float *out,
                             const float2 *otf, float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  auto *fn = cls < kF2dPart[1] ? f2d_launch_p0 : cls < kF2dPart[2] ? f2d_launch_p1 : cls < kF2dPart[3] ? f2d_launch_p2
                                                                                                     : f2d_launch_p3;
  return fn(cls, mode, st, n, n_ch, desc, path, tw, list, in, out, otf, otf_out, mask, ep);
}

// The fused convolutions of every side class in the view (or the PSF's full
// lists): CONV writes the n_ch valid images, CHI2 (one channel) writes the
// chi^2 partials, CORR the adjoint onto the padded grid.
hipError_t launch_fft2d(hipStream_t st, const gf_batch *b, const gf_psf *p, int mode, const float *in, int n_ch,
                        float *out, const int *mask, const WorkView *v, const Chi2Epi *ep) {
  const bool view = v && v->f2d;
  const Work *list = view ? v->f2d : p->d_f2d;
  const int *first = view ? v->f2d_first : p->f2d_first;
  const Chi2Epi e = ep ? *ep : Chi2Epi{};
  for (int c = 0; c < kF2dN; ++c) {
    const int n = first[c + 1] - first[c];
    if (n == 0) continue;
    ProfScope ps(st, mode == MODE_CHI2 ? "k_fft2d_chi2" : mode == MODE_CORR ? "k_fft2d_corr" : "k_fft2d");
    const hipError_t r = f2d_launch(c, mode, st, n, mode == MODE_CHI2 ? 1 : n_ch, b->d_desc, p->d_path,
                                    p->d_tw + p->f2d_tw[c], list + first[c], in, out, p->d_otf, nullptr, mask, e);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

// OTFs of the fused-path PSFs: list holds one stamp per distinct PSF, grouped
// by side class (first[c] .. first[c + 1]).
hipError_t launch_fft2d_otf(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *taps, const Work *list,
                            const int *first) {
  for (int c = 0; c < kF2dN; ++c) {
    const int n = first[c + 1] - first[c];
    if (n == 0) continue;
    const hipError_t r = f2d_launch(c, MODE_OTF, st, n, 1, b->d_desc, p->d_path, p->d_tw + p->f2d_tw[c],
                                    list + first[c], taps, nullptr, nullptr, p->d_otf, nullptr, Chi2Epi{});
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

}  // namespace gf

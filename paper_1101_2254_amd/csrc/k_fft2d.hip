// k_fft2d.hip -- host launchers of the one-workgroup FFT convolution
// (kernels in fft2d_impl.h, built per LDS bucket by k_fft2d_b0 .. b4).
#include "fft2d_impl.h"

namespace gf {

static hipError_t f2d_launch(int bucket, int mode, hipStream_t st, int n, int n_ch, const StampDesc *desc,
                             const PathDesc *path, const float2 *tw_all, const Work *list, const float *in,
                             float *out, const float2 *otf, float2 *otf_out, const int *mask, const Chi2Epi &ep) {
  static decltype(&f2d_launch_b0) const fn[kF2dBuckets] = {f2d_launch_b0, f2d_launch_b1, f2d_launch_b2,
                                                           f2d_launch_b3, f2d_launch_b4};
  return fn[bucket](mode, st, n, n_ch, desc, path, tw_all, list, in, out, otf, otf_out, mask, ep);
}

// The fused convolutions of every bucket in the view (or the PSF's full
// lists): CONV writes the n_ch valid images, CHI2 (one channel) writes the
// chi^2 partials, CORR the adjoint onto the padded grid.  bst: a stream per
// bucket (null: all on st).
hipError_t launch_fft2d(hipStream_t st, const gf_batch *b, const gf_psf *p, int mode, const float *in, int n_ch,
                        float *out, const int *mask, const WorkView *v, const Chi2Epi *ep, const hipStream_t *bst) {
  const bool view = v && v->f2d;
  const Work *list = view ? v->f2d : p->d_f2d;
  const int *first = view ? v->f2d_first : p->f2d_first;
  const Chi2Epi e = ep ? *ep : Chi2Epi{};
  if (first[kF2dBuckets] == first[0]) return hipSuccess;
  // one timing record per call (all buckets)
  ProfScope ps(st, mode == MODE_CHI2 ? "k_fft2d_chi2" : mode == MODE_CORR ? "k_fft2d_corr" : "k_fft2d");
  for (int k = 0; k < kF2dBuckets; ++k) {
    const int n = first[k + 1] - first[k];
    if (n == 0) continue;
    const hipError_t r = f2d_launch(k, mode, bst ? bst[k] : st, n, mode == MODE_CHI2 ? 1 : n_ch, b->d_desc, p->d_path, p->d_tw,
                                    list + first[k], in, out, p->d_otf, nullptr, mask, e);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

// OTFs of the fused-path PSFs: list holds one stamp per distinct PSF, grouped
// by bucket (first[k] .. first[k + 1]).
hipError_t launch_fft2d_otf(hipStream_t st, const gf_batch *b, const gf_psf *p, const float *taps, const Work *list,
                            const int *first) {
  for (int k = 0; k < kF2dBuckets; ++k) {
    const int n = first[k + 1] - first[k];
    if (n == 0) continue;
    const hipError_t r = f2d_launch(k, MODE_OTF, st, n, 1, b->d_desc, p->d_path, p->d_tw, list + first[k], taps,
                                    nullptr, nullptr, p->d_otf, nullptr, Chi2Epi{});
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

}  // namespace gf

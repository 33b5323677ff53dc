// noalloc.hip -- step 3 without any allocation: gf_chi2_noalloc keeps its
// per-chunk chi^2 partials in a fixed device array instead of the context
// workspace, for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid it).
#include <mutex>

#include "gf_internal.h"

namespace gf {
hipError_t launch_chi2(hipStream_t, const gf_batch *, const float *, const void *, bool, const float *,
                       const float *, float *, float2 *, unsigned int *, float2 *, const int *);
}

// The partials (one (hi, lo) pair per 4096-pixel chunk): every device the
// library runs on holds its own copy until the process ends.  Host code uses
// only the address looked up per device, never this name.
static __device__ __align__(256) float2 scratch[GF_CHI2_NOALLOC_MAX_CHUNKS];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
float2 *g_scratch[kMaxDevices] = {};   // the array's device address, per device

}  // namespace

namespace gf {

// Looks up the array's address on `device`, which must be current; once per
// device (gf_create calls it).
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<float2 *>(p);
  return hipSuccess;
}

}  // namespace gf

extern "C" gf_status gf_chi2_noalloc(gf_ctx *c, const gf_batch *b, const float *model, const float *theta,
                                     const float *data, const float *weight, float *resid, float *chi2) {
  gf::ProfBind pb_(c);
  if (!c || !b || !model || !theta || !data || !weight || !chi2) {
    if (c) c->err = "gf_chi2_noalloc: null argument";
    return GF_EINVAL;
  }
  if (b->ctx != c) {
    c->err = "gf_chi2_noalloc: batch belongs to another context";
    return GF_EINVAL;
  }
  const int64_t chunks = (int64_t)b->h_pix.size();
  if (chunks > GF_CHI2_NOALLOC_MAX_CHUNKS) {
    c->err = "gf_chi2_noalloc: the batch has " + std::to_string(chunks) + " chunks of 4096 pixels, above the " +
             std::to_string(GF_CHI2_NOALLOC_MAX_CHUNKS) + " its fixed partials array holds (use gf_chi2)";
    return GF_ESHAPE;
  }
  float2 *part = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
  if (!part) {
    c->err = "gf_chi2_noalloc: the partials array of this device was not set up by gf_create";
    return GF_EDEVICE;
  }
  // every slot the pair sums read is written by its chunk first: nothing to clear
  const hipError_t e = gf::launch_chi2(c->stream, b, model, theta, false, data, weight, resid, part, nullptr,
                                       reinterpret_cast<float2 *>(chi2), nullptr);
  if (e != hipSuccess) {
    c->err = std::string("gf_chi2_noalloc: ") + hipGetErrorString(e);
    return GF_EDEVICE;
  }
  return GF_OK;
}

// lines_api.cpp -- host side of the spectral-line family: line batches and the
// model, chi^2 and Levenberg-Marquardt entry points (kernels in k_lines.hip).
#include <new>
#include <string>
#include <vector>

#include "gf_internal.h"

namespace gf {
hipError_t launch_line_model(hipStream_t, const gf_line_batch *, const float *, const float *, int, float *);
hipError_t launch_line_chi2(hipStream_t, const gf_line_batch *, const float *, const float *, int, const float *,
                            const float *, float2 *);
hipError_t launch_line_lm(const hipStream_t *, const gf_line_batch *, const float *, const float *, const float *,
                          double *, const LineLMParams &, gf_lm_result *);
}  // namespace gf

using namespace gf;

namespace {

gf_status lfail(gf_ctx *c, gf_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

#define LINE_TRY(ctx, expr)                                                                                  \
  do {                                                                                                       \
    hipError_t e_ = (expr);                                                                                  \
    if (e_ != hipSuccess) return lfail(ctx, GF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

gf_status check_call(gf_ctx *c, const gf_line_batch *lb, const void *a, const void *b, int S, const char *what) {
  if (!c || !lb || !a || !b) return lfail(c, GF_EINVAL, std::string(what) + ": null argument");
  if (lb->ctx != c) return lfail(c, GF_EINVAL, std::string(what) + ": line batch of another context");
  if (S < 1 || S > GF_MAX_OVERSAMPLE) return lfail(c, GF_EINVAL, std::string(what) + ": oversample out of range");
  return GF_OK;
}

}  // namespace

extern "C" {

gf_status gf_line_batch_create(gf_ctx *c, int n, const int32_t *N, const int32_t *K, const int32_t *n_lines,
                               gf_line_batch **out) {
  if (!c || !out || !N || !K || !n_lines) return lfail(c, GF_EINVAL, "gf_line_batch_create: null argument");
  *out = nullptr;
  if (n < 1) return lfail(c, GF_EINVAL, "gf_line_batch_create: n < 1");
  gf_line_batch *lb = new (std::nothrow) gf_line_batch();
  if (!lb) return lfail(c, GF_ENOMEM, "gf_line_batch_create: host allocation");
  lb->ctx = c;
  lb->n = n;
  lb->h_desc.resize(n);
  for (int s = 0; s < n; ++s) {
    if (N[s] < 1 || K[s] < 1 || K[s] > GF_LINE_MAX_K || (K[s] % 2) == 0 || n_lines[s] < 1 ||
        n_lines[s] > GF_LINE_MAX_LINES) {
      delete lb;
      return lfail(c, GF_ESHAPE, "gf_line_batch_create: spectrum " + std::to_string(s) +
                                     " needs N >= 1, odd K in 1..GF_LINE_MAX_K, 1..GF_LINE_MAX_LINES lines");
    }
    LineDesc &d = lb->h_desc[s];
    d.N = N[s];
    d.K = K[s];
    d.nl = n_lines[s];
    d.pad0 = 0;
    d.data = lb->n_data;
    d.lsf = lb->n_lsf;
    d.par = lb->n_par;
    lb->n_data += N[s];
    lb->n_lsf += K[s];
    lb->n_par += 3 * n_lines[s] + 1;
    lb->has_nl[n_lines[s]] = true;
  }
  if (lb->n_data > 0x7fffffffLL) {
    delete lb;
    return lfail(c, GF_ESHAPE, "gf_line_batch_create: batch too large");
  }
  hipError_t e = hipMalloc((void **)&lb->d_desc, sizeof(LineDesc) * (size_t)n);
  if (e == hipSuccess) e = hipMemcpy(lb->d_desc, lb->h_desc.data(), sizeof(LineDesc) * (size_t)n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    gf_line_batch_destroy(lb);
    return lfail(c, GF_EDEVICE, std::string("gf_line_batch_create: ") + hipGetErrorString(e));
  }
  *out = lb;
  return GF_OK;
}

void gf_line_batch_destroy(gf_line_batch *lb) {
  if (!lb) return;
  if (lb->d_desc) (void)hipFree(lb->d_desc);
  delete lb;
}

gf_status gf_line_batch_offsets(const gf_line_batch *lb, int64_t *data_off, int64_t *lsf_off, int64_t *par_off) {
  if (!lb) return GF_EINVAL;
  for (int s = 0; s <= lb->n; ++s) {
    const bool end = s == lb->n;
    if (data_off) data_off[s] = end ? lb->n_data : lb->h_desc[s].data;
    if (lsf_off) lsf_off[s] = end ? lb->n_lsf : lb->h_desc[s].lsf;
    if (par_off) par_off[s] = end ? lb->n_par : lb->h_desc[s].par;
  }
  return GF_OK;
}

gf_status gf_line_model(gf_ctx *c, const gf_line_batch *lb, const float *lsf, const float *theta, int S,
                        float *out) {
  ProfBind pb_(c);
  gf_status st = check_call(c, lb, lsf, theta, S, "gf_line_model");
  if (st != GF_OK) return st;
  if (!out) return lfail(c, GF_EINVAL, "gf_line_model: null output");
  LINE_TRY(c, launch_line_model(c->stream, lb, lsf, theta, S, out));
  return GF_OK;
}

gf_status gf_line_chi2(gf_ctx *c, const gf_line_batch *lb, const float *lsf, const float *theta, int S,
                       const float *data, const float *weight, float *chi2) {
  ProfBind pb_(c);
  gf_status st = check_call(c, lb, lsf, theta, S, "gf_line_chi2");
  if (st != GF_OK) return st;
  if (!data || !weight || !chi2) return lfail(c, GF_EINVAL, "gf_line_chi2: null argument");
  LINE_TRY(c, launch_line_chi2(c->stream, lb, lsf, theta, S, data, weight, (float2 *)chi2));
  return GF_OK;
}

gf_status gf_line_fit_lm(gf_ctx *c, const gf_line_batch *lb, const float *lsf, const float *data,
                         const float *weight, double *theta_io, const gf_lm_opts *opts, gf_lm_result *res) {
  ProfBind pb_(c);
  if (opts && opts->struct_size != (int32_t)sizeof(gf_lm_opts))
    return lfail(c, GF_EINVAL, "gf_line_fit_lm: opts->struct_size differs from sizeof(gf_lm_opts) (initialise with gf_lm_opts_default)");
  gf_lm_opts o;
  if (opts)
    o = *opts;
  else
    gf_lm_opts_default(&o);
  gf_status st = check_call(c, lb, lsf, theta_io, o.oversample, "gf_line_fit_lm");
  if (st != GF_OK) return st;
  if (!data || !weight || !res) return lfail(c, GF_EINVAL, "gf_line_fit_lm: null argument");
  if (o.max_iter < 0 || !(o.lambda0 > 0.0) || !(o.lambda_up > 1.0) || !(o.lambda_down > 1.0) ||
      !(o.lambda_max > 0.0) || !(o.ftol >= 0.0) || !(o.xtol >= 0.0))
    return lfail(c, GF_EINVAL, "gf_line_fit_lm: invalid options");
  LineLMParams prm{o.max_iter, o.oversample, o.lambda0, o.lambda_up, o.lambda_down, o.lambda_max, o.ftol, o.xtol,
                   o.lo, o.hi, o.free_mask};
  // fork onto the side streams after the caller's stream, join back
  for (int i = 0; i < GF_LINE_MAX_LINES; ++i)
    if (!c->side[i]) LINE_TRY(c, hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
  for (int i = 0; i <= GF_LINE_MAX_LINES; ++i)
    if (!c->side_ev[i]) LINE_TRY(c, hipEventCreateWithFlags(&c->side_ev[i], hipEventDisableTiming));
  ProfScope ps(c->stream, "k_line_lm");
  LINE_TRY(c, hipEventRecord(c->side_ev[0], c->stream));
  for (int i = 0; i < GF_LINE_MAX_LINES; ++i) LINE_TRY(c, hipStreamWaitEvent(c->side[i], c->side_ev[0], 0));
  LINE_TRY(c, launch_line_lm(c->side, lb, lsf, data, weight, theta_io, prm, res));
  for (int i = 0; i < GF_LINE_MAX_LINES; ++i) {
    LINE_TRY(c, hipEventRecord(c->side_ev[i + 1], c->side[i]));
    LINE_TRY(c, hipStreamWaitEvent(c->stream, c->side_ev[i + 1], 0));
  }
  return GF_OK;
}

}  // extern "C"

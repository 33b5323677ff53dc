/*
 * gf.h -- C ABI of the MI355X galaxy-fitting hot path.
 *
 * Barsdell, Barnes & Fluke, "Fitting Galaxies on GPUs", Sec. 2 describe the
 * fitting loop as five steps: (1) evaluate the model on a grid from the
 * current parameters, (2) convolve it with the PSF, (3) compare model and
 * observation, (4) adjust the parameters, (5) test for completion.  Sec. 3
 * identifies steps 1-3 as transform, FFT (+ transform) and transform + reduce,
 * common to most fitting routines, and argues that the image should stay in
 * device memory for all iterations with only O(1) results going back.  This
 * library implements steps 1-3 as separate calls, their derivatives, and a
 * whole device-resident Levenberg-Marquardt loop (steps 4-5).
 *
 * Conventions for every call:
 *   - Pointers named as device pointers are caller-owned device memory (for
 *     example a torch tensor's data_ptr()); the library never frees them.
 *     Host arrays are copied before the call returns.
 *   - Images are FP32, row-major.  Batches are flat: stamp s occupies the
 *     offsets reported by gf_batch_offsets() in each flat array.
 *   - Work is enqueued on the context's stream (gf_set_stream) and runs
 *     asynchronously; argument and shape errors are detected on the host and
 *     returned before anything is enqueued.  A failure of an earlier
 *     asynchronous launch surfaces as GF_EDEVICE from a later call.
 *   - No C++ exception crosses this boundary.  gf_last_error() returns a
 *     message for the last non-GF_OK status of a context.
 *   - A context is not thread-safe; use one per host thread.
 *
 * Model (the readings the paper leaves open, fixed here):
 *   - parameters per component: x0, y0, Ie, Re, n, q, phi; one sky per stamp;
 *     P = 7 * n_comp + 1 floats per stamp.  phi is in radians, counter-
 *     clockwise from +x (x runs along columns); q = b/a in (0, 1].
 *   - surface brightness: Ie exp(-b_n [(R/Re)^(1/n) - 1]) with
 *     R^2 = x'^2 + y'^2 / q^2, (x', y') the offsets rotated by phi, and b_n the
 *     root of P(2n, b_n) = 1/2 (P the regularised lower incomplete gamma).
 *   - pixel (row i, col j) is centred on (x = j, y = i); its value is the mean
 *     over S x S sub-samples at x = j + (s + 1/2)/S - 1/2 (same for y).
 *   - the model of an H x W stamp with a K x K PSF (K odd, c = (K-1)/2) is
 *     evaluated on a padded grid of Mh x Mw = (H+K-1) x (W+K-1) pixels that
 *     starts at stamp pixel (-c, -c); the convolution keeps the "valid" part
 *       out[y][x] = sum_{u,v} psf[u][v] pad[y+K-1-u][x+K-1-v]
 *     and the sky is added after it.  chi^2 = sum w (d - m)^2.
 */
#ifndef GF_H
#define GF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx gf_ctx;
typedef struct gf_batch gf_batch;
typedef struct gf_psf gf_psf;
typedef struct gf_cnn gf_cnn;

typedef enum {
  GF_OK = 0,
  GF_EINVAL = 1,    /* null pointer or out-of-range argument */
  GF_ESHAPE = 2,    /* sizes that the library does not support or that disagree */
  GF_ENOMEM = 3,    /* device or host allocation failed */
  GF_EDEVICE = 4,   /* a HIP call or an earlier asynchronous launch failed */
  GF_ENUMERIC = 5,  /* non-finite input where a finite value is required */
  GF_ENOTCONV = 6   /* per-stamp LM status: stopped without meeting ftol/xtol */
} gf_status;

#define GF_NPC 7           /* parameters per Sersic component */
#define GF_MAX_COMP 4      /* components per stamp */
#define GF_MAX_K 129       /* largest PSF side */
#define GF_MAX_FFT 2048    /* largest FFT side; stamps need H+K-1, W+K-1 <= this */
#define GF_MAX_OVERSAMPLE 8
#define GF_LINE_MAX_K 65       /* longest line-spread function (odd) */
#define GF_LINE_MAX_LINES 3    /* Gaussian lines per spectrum */

/* Convolution path of a prepared PSF. */
#define GF_CONV_AUTO 0     /* chosen per stamp from the PSF and grid size */
#define GF_CONV_FFT 1      /* Fourier-space product (Sec. 3, step 2); one-workgroup form
                              where the side allows it, else multi-pass */
#define GF_CONV_DIRECT 2   /* direct sum over taps */
#define GF_CONV_FFT_MULTIPASS 3  /* Fourier-space product, multi-pass form for every stamp */
#define GF_CONV_FFT_FUSED 4      /* Fourier-space product, one-workgroup form for every stamp
                                    (GF_ESHAPE when a side L exceeds GF_FFT_FUSED_MAX) */
#define GF_FFT_FUSED_MAX 192     /* largest side of the one-workgroup form */

/* gf_jacobian modes. */
#define GF_JAC_FULL 0      /* d m / d theta images */
#define GF_JAC_ADJOINT 1   /* vector-Jacobian product sum_i c_i d m_i / d theta */

/* ------------------------------------------------------------- contexts */

/* Create a context on HIP device `device`; builds the b_n table (FP64 on the
 * host, FP32 on the device).  *ctx is set to NULL on failure.
 * autotune_cache: path of the context's tuning file (nullable).  With a
 * path, the table it holds for this GPU (architecture and device name) is
 * loaded, and gf_psf_prepare(GF_CONV_AUTO) measures every one-workgroup FFT
 * side it meets that the table lacks (see gf_tune_form_get; this launches
 * timing convolutions and allocates temporary device memory in that call)
 * and rewrites the file.  A later context reading the same file takes the
 * same choices, so its results are the same bits.  Without a path nothing
 * is measured and untuned sides take the default rule.
 * The context also creates three non-blocking streams (default priority) on
 * which the one-workgroup FFT launches of a convolution run beside its
 * multi-pass launches, joined to the calling stream by events before the
 * call returns (and recorded into the LM iteration graphs). */
gf_status gf_create(gf_ctx **ctx, int device, const char *autotune_cache);
void gf_destroy(gf_ctx *ctx);
/* Tuning table of the context, read by gf_psf_prepare(GF_CONV_AUTO) and
 * gf_fit_lm.  For an FFT side L of the one-workgroup form (an even
 * 2^a 3^b 5^c <= GF_FFT_FUSED_MAX):
 *   form: the FFT form the automatic choice takes for that side: 1
 *     multi-pass, 2 one-workgroup, -1 untuned (then one-workgroup up to 160,
 *     multi-pass above);
 *   min_active: per group of sides of similar on-chip size (up to 64, 96,
 *     128, 160 and 192), the fewest still-fitting stamps of that group for
 *     which gf_fit_lm keeps them on the one-workgroup form; when fewer
 *     remain (checked when it restricts its launches to the unfinished
 *     stamps) they move to the multi-pass form for the rest of the fit.
 *     0 keeps them always.
 * Both forms give the same convolution to rounding (a fit whose stamps
 * move may take other last bits).  The getters return 0 (form) or -1
 * (min_active) for sides that are not one-workgroup sides; the setters
 * return GF_EINVAL for them.
 * direct_max_k: GF_CONV_AUTO convolves PSFs of side K <= direct_max_k on
 * the direct path and larger ones by FFT (default 7; measured by
 * gf_autotune with no sides, or on the first gf_psf_prepare(GF_CONV_AUTO)
 * of a context with a tuning file that meets a PSF side in 3..15). */
/* Measure the FFT forms of the given one-workgroup sides now (NULL and 0:
 * every one of them, and the direct-path threshold): per side, 256 stamps
 * of padded side L convolved in seven channels by each form, the faster
 * form kept; for the threshold, 256 stamps of 64 x 64 convolved in seven
 * channels directly and by FFT for K = 3, 5, ..., 15, direct_max_k the
 * largest K up to which the direct path is not slower.  Writes the
 * context's tuning file when it has one (min_active values set on the
 * context are written too).  GF_EINVAL for a side that is not a
 * one-workgroup side. */
gf_status gf_autotune(gf_ctx *ctx, const int32_t *sides, int n_sides);
int gf_tune_form_get(const gf_ctx *ctx, int L);
gf_status gf_tune_form_set(gf_ctx *ctx, int L, int form);
int gf_tune_min_active_get(const gf_ctx *ctx, int L);
gf_status gf_tune_min_active_set(gf_ctx *ctx, int L, int n);
int gf_tune_direct_get(const gf_ctx *ctx);
gf_status gf_tune_direct_set(gf_ctx *ctx, int direct_max_k);   /* 1..GF_MAX_K, odd (GF_EINVAL otherwise) */

/* All later work of this context is enqueued on `hip_stream` (a hipStream_t;
 * NULL = the default stream). */
gf_status gf_set_stream(gf_ctx *ctx, void *hip_stream);
const char *gf_last_error(const gf_ctx *ctx);
/* Block until all work enqueued by this context has finished; returns
 * GF_EDEVICE if any of it failed. */
gf_status gf_synchronize(gf_ctx *ctx);

/* --------------------------------------------------------------- batches */

/* Describe n_stamps stamps (host arrays, copied): stamp s is H[s] x W[s]
 * pixels, has a K[s] x K[s] PSF (K odd) and n_comp[s] components.
 * shared_image != 0 declares that every stamp shares one observation and one
 * PSF (a likelihood batch: many parameter vectors against one image); all
 * stamps must then have the same H, W, K and n_comp, and data/weight/psf
 * arrays hold a single image.  Errors: GF_EINVAL (also for n_stamps < 1: a
 * batch holds at least one stamp), GF_ESHAPE (K even or above GF_MAX_K,
 * padded side above GF_MAX_FFT, n_comp outside 1..GF_MAX_COMP). */
gf_status gf_batch_create(gf_ctx *ctx, int n_stamps, const int32_t *H, const int32_t *W, const int32_t *K,
                          const int32_t *n_comp, int shared_image, gf_batch **out);
void gf_batch_destroy(gf_batch *batch);

/* A batch whose stamps come in observation groups (several fits of one
 * galaxy, e.g. from different starting points or with different numbers of
 * components): group[s] in 0 .. G-1, every id used.  All stamps of a group
 * share one observation (data and weight) and one PSF, so they need the
 * same H, W and K; n_comp may differ.  Group g's image sits at offset
 * sum_{g' < g} H_g' W_g' of the data and weight arrays and its PSF at
 * sum_{g' < g} K_g'^2 of the taps (gf_batch_offsets reports these per
 * stamp); per-stamp arrays (models, parameters) are laid out as usual.
 * gf_psf_prepare computes one OTF per group. */
gf_status gf_batch_create_grouped(gf_ctx *ctx, int n_stamps, const int32_t *H, const int32_t *W, const int32_t *K,
                                  const int32_t *n_comp, const int32_t *group, gf_batch **out);
/* Number of observation groups (G for grouped batches, 1 for shared-image
 * batches, n_stamps otherwise). */
int gf_batch_groups(const gf_batch *batch);

/* Flat array sizes (elements) for a batch; any output may be NULL.
 *   n_pix: sum H*W        (model, residual images)
 *   n_pad: sum Mh*Mw      (padded model grids, per channel)
 *   n_psf: sum K*K        (PSF taps; K*K when shared)
 *   n_par: sum P          (parameters)
 *   n_img: n_pix, or H*W when shared (data, weight)
 *   n_jac: sum P*H*W      (full Jacobian images) */
gf_status gf_batch_sizes(const gf_batch *batch, int64_t *n_pix, int64_t *n_pad, int64_t *n_psf, int64_t *n_par,
                         int64_t *n_img, int64_t *n_jac);
/* Per-stamp offsets (host arrays of n_stamps int64, any may be NULL) into
 * the flat arrays above. */
gf_status gf_batch_offsets(const gf_batch *batch, int64_t *pix, int64_t *pad, int64_t *psf, int64_t *par,
                           int64_t *img, int64_t *jac);
int gf_batch_count(const gf_batch *batch);

/* ------------------------------------------------------------------ PSF */

/* Prepare the PSF of every stamp (device array of n_psf floats, taps used as
 * given: normalise them beforehand if unit sum is wanted).  For stamps on the
 * FFT path this computes the optical transfer function on an L x L grid
 * (L = smallest even 2^a 3^b 5^c >= the padded side) on the device; the
 * prepared object owns that memory.  `mode` is one of the GF_CONV_* values.
 * The FFT path comes in two forms that compute the same convolution:
 *   one-workgroup (L <= GF_FFT_FUSED_MAX): a workgroup holds a whole
 *     channel's 2-D spectrum in on-chip memory (the paper's all-to-all FFT
 *     step without a trip through device memory);
 *   multi-pass: row, column and inverse-row launches with the spectra in
 *     device memory, for any L.
 * GF_CONV_AUTO takes the direct sum for K <= 7 and the FFT otherwise, in the
 * form the context's tuning table names for that side (gf_create), else the
 * one-workgroup form where it applies.  The psf array must stay valid while
 * *out is used. */
gf_status gf_psf_prepare(gf_ctx *ctx, const gf_batch *batch, const float *psf, int mode, gf_psf **out);
void gf_psf_destroy(gf_psf *psf);
/* Host arrays of n_stamps ints (either may be NULL): uses_fft[s] = 0 for the
 * direct sum, 1 for the multi-pass FFT, 2 for the one-workgroup FFT;
 * fft_side[s] = L (0 on the direct path). */
gf_status gf_psf_paths(const gf_psf *psf, int32_t *uses_fft, int32_t *fft_side);

/* ------------------------------------------------------ step 1: evaluate */

/* Paper Sec. 2 step 1 / Sec. 3 item 1 (a per-pixel transform).  theta:
 * device [n_par] FP32.  Writes model_pad (device [n_pad]): the sum of all
 * components, mean of oversample^2 sub-samples, no sky.  oversample in
 * 1..GF_MAX_OVERSAMPLE. */
gf_status gf_eval_model(gf_ctx *ctx, const gf_batch *batch, const float *theta, int oversample, float *model_pad);

/* ----------------------------------------------------- step 2: convolve */

/* Paper Sec. 2 step 2 / Sec. 3 item 2 (FFT + pointwise transform).  in:
 * device, n_ch channels per stamp; stamp s, channel c starts at
 * pad_off[s]*n_ch + c*Mh*Mw.  out: device; stamp s, channel c starts at
 * pix_off[s]*n_ch + c*H*W.  n_ch in 1..64. */
gf_status gf_convolve_psf(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *in, int n_ch,
                          float *out);

/* Steps 1-2 plus sky: out (device [n_pix]) = conv(components) + sky, the
 * model image that step 3 compares with the observation.  work as in
 * gf_likelihood (NULL = context workspace). */
gf_status gf_model(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *theta, int oversample,
                   float *out, void *work);

/* ------------------------------------------------------- step 3: compare */

/* Paper Sec. 2 step 3 / Sec. 3 item 3 (transform + reduce: the sum of squared
 * differences).  model: device [n_pix] convolved model without sky; the sky
 * is read from theta (device [n_par]).  data, weight: device [n_img]
 * (weight = inverse variance, 0 masks a pixel).  resid (nullable): device
 * [n_pix] = sqrt(w) (d - m - sky).  chi2: device [2 * n_stamps], an FP32
 * (hi, lo) pair per stamp whose exact sum is the compensated chi^2.  The
 * reduction order is fixed, so results are bitwise reproducible. */
gf_status gf_chi2(gf_ctx *ctx, const gf_batch *batch, const float *model, const float *theta, const float *data,
                  const float *weight, float *resid, float *chi2);

/* gf_chi2 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and the same bits as gf_chi2, with the per-chunk
 * partials in a fixed array of GF_CHI2_NOALLOC_MAX_CHUNKS (hi, lo) pairs
 * (1 MiB) that the library holds on each device from gf_create until the
 * process ends, instead of the context workspace.  It allocates nothing and
 * calls no allocating routine.  A batch with more than
 * GF_CHI2_NOALLOC_MAX_CHUNKS chunks of 4096 pixels (about 5.4e8 pixels) is
 * refused with GF_ESHAPE before anything is enqueued.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other contexts, other threads) race and must be ordered by the caller. */
#define GF_CHI2_NOALLOC_MAX_CHUNKS 131072
gf_status gf_chi2_noalloc(gf_ctx *ctx, const gf_batch *batch, const float *model, const float *theta,
                          const float *data, const float *weight, float *resid, float *chi2);

/* Steps 1-3 in one call: chi2 (device [2 * n_stamps], (hi, lo) pairs as in
 * gf_chi2) of every stamp at theta (device [n_par] FP32).  work: device
 * scratch of at least gf_likelihood_workspace() bytes, or NULL to use the
 * context's own workspace (which then grows on the first call). */
gf_status gf_likelihood(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *theta, int oversample,
                        const float *data, const float *weight, float *chi2, void *work);
int64_t gf_likelihood_workspace(const gf_batch *batch, const gf_psf *psf);

/* ------------------------------------------------------- derivatives */

/* Derivatives of the model m = conv(components) + sky.
 * GF_JAC_FULL: out = device [n_jac]; stamp s holds P images of H*W,
 *   d m / d theta_p, the last one (sky) all ones.  cot, weight ignored.
 * GF_JAC_ADJOINT: out = device [n_par];
 *   out[p] = scale * sum_i cot_i * (weight ? sqrt(weight_i) : 1) * d m_i / d theta_p
 *   computed by correlating the cotangent with the PSF and contracting it
 *   with the point derivatives on the padded grid (no Jacobian images).
 *   With cot = resid from gf_chi2 and scale = -2 this is d chi^2 / d theta.
 * The derivative of b_n in n comes from the same table as b_n. */
gf_status gf_jacobian(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *theta, int oversample,
                      int mode, const float *cot, const float *weight, float scale, float *out);

/* ----------------------------------------------- steps 4-5: LM fitting */

typedef struct {
  int32_t struct_size;  /* sizeof(gf_lm_opts): set by gf_lm_opts_default, checked by every call that
                           takes the struct (GF_EINVAL otherwise), so a caller built against a
                           header with another layout is refused instead of misread */
  int32_t max_iter;     /* iteration cap (default 100) */
  int32_t oversample;   /* S (default 5) */
  double lambda0;       /* initial damping (1e-3) */
  double lambda_up;     /* factor on a rejected step (10) */
  double lambda_down;   /* divisor on an accepted step (10) */
  double lambda_max;    /* give up above this (1e10) */
  double ftol;          /* stop when (chi2 - chi2')/chi2' < ftol on an accepted step (1e-5) */
  double xtol;          /* stop when max |dtheta_i| / max(|theta_i|, 1) < xtol on an accepted step (1e-10) */
  const double *lo;     /* device [n_par] lower bounds or NULL */
  const double *hi;     /* device [n_par] upper bounds or NULL */
  const uint8_t *free_mask; /* device [n_par], nonzero = fitted, or NULL = all free */
  int32_t poll_every;   /* iterations between host checks of the active-stamp count (default 4) */
  int32_t use_graph;    /* capture one iteration in a HIP graph and replay it (default 1) */
  int32_t speculate;    /* evaluate the Jacobian together with every trial point instead of after
                           acceptance: 1 on, 0 off, -1 (default) on for single-stamp batches */
  const double *start;  /* device [n_par] start point, or NULL (default): theta_io holds it.  When
                           set, theta_io is output only and start is not written; the two are the
                           same buffer or do not overlap. */
} gf_lm_opts;

typedef struct {
  double chi2;     /* chi^2 at the returned parameters */
  double lambda;   /* damping at exit */
  int32_t iters;   /* iterations taken */
  int32_t nfev;    /* model evaluations (steps 1-3): the start point and every trial */
  int32_t njev;    /* Jacobians that enter a solve (with speculate, every trial also evaluates
                      one, from which its model comes) */
  int32_t status;  /* GF_OK (converged) or GF_ENOTCONV */
  int32_t reason;  /* 1 ftol, 2 xtol, 3 chi2 = 0, 4 lambda above lambda_max, 5 iteration cap */
  int32_t pad;
} gf_lm_result;

/* Fills every field with its default, struct_size included.  Initialise the
 * struct with this call and then change fields. */
void gf_lm_opts_default(gf_lm_opts *opts);

/* Levenberg-Marquardt over every stamp of the batch at once (Marquardt 1963;
 * the paper's galfit route for step 4).  Per stamp and iteration:
 *   A = J^T W J, g = J^T W (d - m) over the free parameters,
 *   (A + lambda diag(max(A_ii, 1e-12 max A_jj))) delta = g  by FP64 Cholesky
 *   (not positive definite: lambda *= up, try again),
 *   theta' = clip(theta + delta, lo, hi); accept iff chi2(theta') < chi2(theta)
 *   (lambda /= down), else reject (lambda *= up).
 * theta_io: device [n_par] FP64, start in (unless opts->start gives it), best accepted
 * point out.
 * With speculate the trial point's model comes from its Jacobian images
 * (the model is linear in each Ie: m = sky + sum_c Ie_c dm/dIe_c), so an
 * accepted step already has the next normal equations; a rejected one has
 * spent a Jacobian instead of one model.  This pays where launches are
 * latency-bound (one large image), not in large batches with many
 * rejections.  The steps taken are the same rule either way; chi^2 values
 * differ in the last bits.
 * res: device [n_stamps].  data, weight: device [n_img].  All iterations run
 * on the device; the host only reads the count of still-active stamps every
 * poll_every iterations.  Stamps that finish stop costing work.
 * The fit runs on streams of the context, ordered after and before the
 * caller's stream by events; a batch of 512 or more stamps in the plain form
 * runs as two halves on two of them, each polled every poll_every
 * iterations.  A stamp runs the same kernels as in one batch; only the
 * iteration at which a one-workgroup FFT stamp moves to the multi-pass
 * launches (once few stamps of its size are left) follows its half's count,
 * which can change the last bits of its result.
 * Returns GF_OK when the call ran (per-stamp outcomes are in res).  Data or
 * weights that are not finite make that stamp's chi^2 non-finite: its fit
 * then rejects every step and ends with GF_ENOTCONV, reason 4, at the
 * (clipped) start; mask bad pixels with weight 0 and a finite data value. */
gf_status gf_fit_lm(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *data, const float *weight,
                    double *theta_io, const gf_lm_opts *opts, gf_lm_result *res);

/* Best fit per observation group after gf_fit_lm: the member with the
 * lowest chi^2 among those with status GF_OK (among all members if none
 * converged); ties go to the lowest stamp index and NaN never wins.
 * res: device [n_stamps] from gf_fit_lm; theta: device [n_par] FP64 (the
 * fitted parameters); best: device FP64 [n_groups][29] (the winner's P
 * parameters, then zeros); best_stamp: device int32 [n_groups] or null. */
gf_status gf_group_best(gf_ctx *ctx, const gf_batch *batch, const gf_lm_result *res, const double *theta,
                        double *best, int32_t *best_stamp);

/* Multi-start set for single-Sersic stamps (P = 8): out[g * n_starts + k] =
 * theta0[g] changed by rule k: 0 none; 1 n = 1 (exponential), Re x 1.5;
 * 2 n = 4 (de Vaucouleurs), Re x 0.7; 3 phi + pi/2 (the other axis), mod pi.
 * theta0: device [n_groups][8] FP64; out: device [n_groups * n_starts][8];
 * 1 <= n_starts <= 4.  With gf_batch_create_grouped (group = g for the
 * stamps g * n_starts .. + n_starts - 1), gf_fit_lm and gf_group_best this
 * is the multi-start fit. */
gf_status gf_expand_starts(gf_ctx *ctx, int n_groups, int n_starts, const double *theta0, double *out);

/* ------------------------------------------------------------ downhill simplex
 *
 * Nelder & Mead (1965) over every stamp of the batch at once: the paper's
 * other step-4 route (Sec. 2), on the same steps 1-3.  Per stamp a simplex
 * of P + 1 vertices (x0 and x0 + step_j e_j) moves by reflection (1),
 * expansion (2), contraction (1/2) and shrink (1/2) steps; points are
 * clipped into [lo, hi]; ties in the ordering go to the lower index for the
 * best vertex and to the higher for the worst.  A stamp stops when
 * 2 (f_w - f_b) <= ftol (|f_w| + |f_b|) + 1e-300, or after max_iter
 * iterations.  Each device iteration evaluates one candidate per active
 * stamp; the host reads the active count every poll_every iterations.
 * theta_io: device [n_par] start in, best vertex out.  res: device
 * [n_stamps] (chi2 of the best vertex, iterations, evaluations, status;
 * lambda and njev are 0).  trace: device FP64 [n_stamps][trace_cap] or null:
 * chi^2 of every evaluated point of each stamp, in evaluation order (the
 * first trace_cap of them). */
typedef struct {
  int32_t max_iter;     /* default 2000 */
  int32_t oversample;   /* default 5 */
  double ftol;          /* default 1e-8 */
  const double *step;   /* device [n_par]: initial simplex offsets (required) */
  const double *lo;     /* device [n_par] or null */
  const double *hi;     /* device [n_par] or null */
  int32_t poll_every;   /* default 16 */
  int32_t use_graph;    /* default 1 */
} gf_simplex_opts;

void gf_simplex_opts_default(gf_simplex_opts *opts);
gf_status gf_fit_simplex(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *data,
                         const float *weight, double *theta_io, const gf_simplex_opts *opts, gf_lm_result *res,
                         double *trace, int trace_cap);

/* ------------------------------------------------------------ MCMC
 *
 * The paper names Bayesian sampling (galphat) as the third routine family
 * built on the same steps 1-3 (Sec. 2).  gf_mcmc_run runs random-walk
 * Metropolis with one chain per stamp of the batch (typically a
 * shared-image batch: many chains on one observation):
 *   target    exp(-chi2(theta)/2), flat prior on [lo, hi] (null: unbounded);
 *   proposal  theta' = theta + scale * z, z ~ N(0, I) per parameter;
 *   accept    iff ln u < -(chi2(theta') - chi2(theta))/2 (theta' outside the
 *             box is rejected without evaluation).
 * Random numbers: Philox4x64-10 with key (key0, key1); chain c at step t uses
 * counter (b, c, step0 + t, stream) with b = 0..3 giving the normals
 * z_{4b..4b+3} (Box-Muller as in gf_normal_noise) and b = 4 word 0 the
 * uniform u.  Running n steps from step0 and then n more from step0 + n gives
 * the same chain as 2n steps at once.
 * theta_io: device [n_par] FP64 start in, last state out.  chi2_out: device
 * [n_stamps] FP64, chi^2 of the last state.  samples: device FP32
 * [n_steps / thin][n_par] (the state after steps thin, 2 thin, ...), or null.
 * accepted: device int32 [n_stamps], incremented per accepted step, or null.
 * All steps run on the device (one captured HIP graph replayed n_steps times). */
typedef struct {
  int32_t n_steps;
  int32_t oversample;
  int32_t thin;
  int32_t use_graph;
  uint64_t key0, key1;
  uint64_t stream;
  int64_t step0;
  const double *scale;  /* device [n_par] proposal standard deviations (null: no move) */
  const double *lo;     /* device [n_par] or null */
  const double *hi;     /* device [n_par] or null */
} gf_mcmc_opts;

void gf_mcmc_opts_default(gf_mcmc_opts *opts);
gf_status gf_mcmc_run(gf_ctx *ctx, const gf_batch *batch, const gf_psf *psf, const float *data, const float *weight,
                      double *theta_io, double *chi2_out, const gf_mcmc_opts *opts, float *samples,
                      int32_t *accepted);

/* ------------------------------------------------------------ starting points
 *
 * The paper's outlook (Sec. 5) notes that a fit only finds the minimum near
 * its starting point and that global strategies help avoid local minima and
 * unphysical results; these calls produce starting points for single-Sersic
 * stamps (P = 8: x0, y0, Ie, Re, n, q, phi, sky) for gf_fit_lm.
 *
 * Default guess (image moments), gf_moments_guess, per stamp of an H x W
 * batch with one component:
 *   sky     = median of the outer 4-pixel frame, s = its RMS about the median;
 *   weights v = (d - sky) * clamp((d - sky)/s - 2, 0, 1)  (a ramp from 2 s to 3 s);
 *   centre  = v-weighted mean of (x, y); q and phi from the v-weighted second
 *             moments (q = sqrt(minor/major eigenvalue), phi = major axis
 *             angle in [0, pi)), q clamped to [0.05, 1];
 *   Re      = elliptical radius (axes q, phi) at which the cumulative v
 *             reaches half of sum(v), linear between neighbouring pixels;
 *   n = 2;  Ie = F / (2 pi n Re^2 q e^{b_n} b_n^{-2n} Gamma(2n)) with
 *             F = sum(d - sky) over the stamp (the flux of a Sersic profile).
 * data: device [n_img]; theta: device [n_par] FP64.  The frame must hold at
 * most 16384 pixels.  Stamps with no positive weight get the stamp centre,
 * Re = 2, q = 1, phi = 0 and Ie from F (at least 1e-3). */
gf_status gf_moments_guess(gf_ctx *ctx, const gf_batch *batch, const float *data, double *theta);

/* Learned proposal (a convolutional network, trained on rendered stamps):
 *   input  side x side stamp, normalised as asinh((d - m) / s) with m, s the
 *          mean and population standard deviation of the outer 4-pixel frame;
 *   4 x [3x3 convolution, stride 2, padding 1, ReLU], channels 32, 32, 64, 64;
 *   dense (side/16)^2*64 -> 256, ReLU, dense 256 -> 8.
 * BF16 operands with FP32 accumulation on the matrix cores; FP32 master
 * weights; mean-squared-error loss; Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 * with bias correction.
 * Parameters in canonical order and layout (gf_cnn_param_count floats):
 *   w1 [32][3][3][1], b1 [32], w2 [32][3][3][32], b2 [32], w3 [64][3][3][32],
 *   b3 [64], w4 [64][3][3][64], b4 [64], w5 [256][(side/16)^2*64] (input
 *   flattened in (y, x, channel) order), b5 [256], w6 [8][256], b6 [8].
 * The object owns its weights, Adam moments and the workspace of max_batch
 * stamps.  side: a multiple of 16 in 16..1024. */
gf_status gf_cnn_create(gf_ctx *ctx, int side, int max_batch, gf_cnn **out);
/* Waits for the device and frees the object (safe after gf_destroy of its context). */
void gf_cnn_destroy(gf_cnn *cnn);
int64_t gf_cnn_param_count(const gf_cnn *cnn);
/* He-uniform weights (bound sqrt(6 / fan_in)) from Philox4x64-10 with key
 * (key, 0x5eed), zero biases; resets Adam. */
gf_status gf_cnn_init(gf_cnn *cnn, uint64_t key);
/* params, out: device, canonical layout.  set_params resets Adam. */
gf_status gf_cnn_set_params(gf_cnn *cnn, const float *params);
gf_status gf_cnn_get_params(gf_cnn *cnn, float *out);
/* stamps: device [n][side][side]; out: device [n][8] network outputs
 * (targets as coded by gf_cnn_encode).  Any n >= 0 (runs in batches). */
gf_status gf_cnn_forward(gf_cnn *cnn, const float *stamps, int n, float *out);
/* Loss and gradients for one batch (1 <= n <= max_batch): targets device
 * [n][8]; grads device canonical layout (nullable); loss device float
 * (nullable), the mean over the n x 8 outputs. */
gf_status gf_cnn_gradients(gf_cnn *cnn, const float *stamps, const float *targets, int n, float *grads, float *loss);
/* gf_cnn_gradients followed by one Adam step with learning rate lr. */
gf_status gf_cnn_train_step(gf_cnn *cnn, const float *stamps, const float *targets, int n, float lr, float *loss);
/* Number of Adam steps taken since the last init / set_params. */
int64_t gf_cnn_steps(const gf_cnn *cnn);
/* Parameter coding of a side-N stamp (theta device [n][8] FP32 in, targets
 * device [n][8] out):
 *   t0 = x0 - N/2, t1 = y0 - N/2, t2 = (ln Ie - a)/b over Ie in [0.5, 5],
 *   t3 = (ln Re - a)/b over Re in [2, N/4] (a, b: midpoint and half-width of
 *   the log range), t4 = (n - 3.25)/2.75, (t5, t6) = (1 - q)(cos 2phi, sin 2phi)/0.8,
 *   t7 = (sky - 0.025)/0.025.
 * gf_cnn_decode inverts it into FP64 theta, clamping n to [0.2, 10] and
 * 1 - q to [0, 0.95], phi to [0, pi). */
gf_status gf_cnn_encode(gf_ctx *ctx, int n, int side, const float *theta, float *targets);
gf_status gf_cnn_decode(gf_ctx *ctx, int n, int side, const float *targets, double *theta);

/* ------------------------------------------------------------ random numbers
 * Philox4x64-10 (Salmon et al., SC 2011): block b uses the 256-bit counter
 * counter + b (counter: host [4], word 0 least significant; null = zero)
 * and the key (key0, key1).
 * gf_philox: out device [n_blocks][4] raw words.
 * gf_normal_noise: out[j] = clean[j] + sigma z_j (clean nullable = 0);
 *   z_{4b..4b+3} come from block b by Box-Muller on 24-bit uniforms
 *   u = (w >> 40 + 1/2) 2^-24: (u0, u1) -> sqrt(-2 ln u0)(cos 2pi u1, sin 2pi u1),
 *   (u2, u3) likewise; computed in FP64, stored FP32.  out may equal clean.
 * gf_draw_prior: theta device [n][8] FP32, stamp i from blocks 2i, 2i+1
 *   (uniforms u0..u7): n = 0.5 + 5.5 u0, Re = 2 + (N/4 - 2) u1,
 *   q = 0.2 + 0.8 u2, phi = pi u3, Ie = 0.5 * 10^u4, x0 = N/2 + 2 u5 - 1,
 *   y0 = N/2 + 2 u6 - 1, sky = 0.05 u7. */
gf_status gf_philox(gf_ctx *ctx, uint64_t key0, uint64_t key1, const uint64_t *counter, int64_t n_blocks,
                    uint64_t *out);
gf_status gf_normal_noise(gf_ctx *ctx, int64_t n, float sigma, uint64_t key0, uint64_t key1, const uint64_t *counter,
                          const float *clean, float *out);
gf_status gf_draw_prior(gf_ctx *ctx, int n, int side, uint64_t key0, uint64_t key1, const uint64_t *counter,
                        float *theta);

/* ------------------------------------------------------------ profiling */

/* Per-kernel timing: while enabled, every kernel launch of this context is
 * bracketed by HIP events recorded on the stream it is launched on (launches
 * inside a captured HIP graph are not timed).  gf_profile_start clears the
 * records; gf_profile_kernels synchronizes the device and returns the number
 * of distinct kernel names; gf_profile_get returns the name, the number of
 * timed launches and their summed duration in milliseconds for index i. */
gf_status gf_profile_start(gf_ctx *ctx);
gf_status gf_profile_stop(gf_ctx *ctx);
int gf_profile_kernels(gf_ctx *ctx);
gf_status gf_profile_get(gf_ctx *ctx, int i, char *name, int name_cap, int64_t *launches, double *total_ms);

/* Roofline calibration probes on the context's device (blocking; they
 * allocate and free their own buffers).
 *   kind 0: streaming triad c = a + s b over n floats per array, reps times;
 *           result = GB/s counting 12 bytes per element.
 *   kind 1: eight independent FP32 FMA chains of n steps per thread (64
 *           workgroups of 256 per compute unit), reps times; result = TFLOP/s.
 *   kind 2: four chains of exp2(log2(x) a) (hardware transcendentals) of n
 *           steps per thread; result = 10^9 transcendental operations/s. */
gf_status gf_probe(gf_ctx *ctx, int kind, int64_t n, int reps, double *result);

/* ------------------------------------------------ spectral-line fitting */

/* The same three steps in one dimension (paper Sec. 5: spectral-line fitting
 * as the next problem for the method once the dimensionality may change).
 * Model of a spectrum of N channels (the readings of the image model, in
 * 1-D): channel i is centred at x = i and is the mean of S sub-samples at
 * x = i + (s + 1/2)/S - 1/2 of  sum_k A_k exp(-(x - mu_k)^2 / (2 sigma_k^2)),
 * evaluated on a padded axis of N + K - 1 channels starting at channel -c
 * (c = (K-1)/2), convolved with the K-tap line-spread function keeping the
 * valid part  out[i] = sum_u lsf[u] pad[i + K - 1 - u],  plus a constant
 * continuum.  Parameters per spectrum: [A, mu, sigma] per line (mu, sigma in
 * channels), then the continuum: P = 3 n_lines + 1.  chi^2 = sum w (d - m)^2.
 *
 * A line batch holds n spectra of uneven N (>= 1), odd K (1..GF_LINE_MAX_K)
 * and 1..GF_LINE_MAX_LINES lines each.  Flat layouts: spectrum s's data,
 * weight and model occupy [data_off[s], data_off[s+1]), its LSF taps
 * [lsf_off[s], lsf_off[s+1]), its parameters [par_off[s], par_off[s+1]). */
typedef struct gf_line_batch gf_line_batch;

gf_status gf_line_batch_create(gf_ctx *ctx, int n, const int32_t *N, const int32_t *K, const int32_t *n_lines,
                               gf_line_batch **out);
void gf_line_batch_destroy(gf_line_batch *lb);
/* Host arrays of n + 1 offsets each (any may be NULL). */
gf_status gf_line_batch_offsets(const gf_line_batch *lb, int64_t *data_off, int64_t *lsf_off, int64_t *par_off);

/* Steps 1-2 plus continuum: out (device [n_data]) = the model spectra.
 * lsf: device [n_lsf]; theta: device [n_par] FP32; oversample 1..8. */
gf_status gf_line_model(gf_ctx *ctx, const gf_line_batch *lb, const float *lsf, const float *theta, int oversample,
                        float *out);

/* Steps 1-3: chi2 (device [2 n]) compensated (hi, lo) FP32 pairs as in
 * gf_chi2; data, weight: device [n_data]. */
gf_status gf_line_chi2(gf_ctx *ctx, const gf_line_batch *lb, const float *lsf, const float *theta, int oversample,
                       const float *data, const float *weight, float *chi2);

/* Levenberg-Marquardt over every spectrum with the rule of gf_fit_lm (opts:
 * max_iter, oversample, lambda0/up/down/max, ftol, xtol, lo, hi, free_mask
 * as there; poll_every and use_graph are unused).  One workgroup per
 * spectrum runs all of that spectrum's iterations in a single launch.
 * theta_io: device [n_par] FP64, start in, best accepted point out;
 * res: device [n]. */
gf_status gf_line_fit_lm(gf_ctx *ctx, const gf_line_batch *lb, const float *lsf, const float *data,
                         const float *weight, double *theta_io, const gf_lm_opts *opts, gf_lm_result *res);

/* ---------------------------------------------------- data-cube fitting */

/* The same three steps in three dimensions (paper Sec. 5: cube fitting as a
 * problem for the method once the dimensionality may change; the model is a
 * reading).  Cube s holds Nc spectral channels of an H_s x W_s image,
 * channel-major [c][y][x]; channel c is centred at v = c (velocities in
 * channel units), spaxel (i, j) at (x = j, y = i).  Its model is one Sersic
 * component (the image model's profile and geometry) whose light carries a
 * Gaussian emission line of width sigma_v centred at the line-of-sight
 * velocity of a thin rotating disk with the component's geometry,
 *   V(x, y) = v0 + vproj (2/pi) atan(R/rt) x'/R   (V = v0 at R = 0),
 * x' the offset along the major axis, R the elliptical radius, vproj the
 * projected rotation amplitude and rt the turnover radius.  A voxel is the
 * mean over S x S spatial and Sv spectral midpoint sub-samples of
 * I(x, y) exp(-(v - V)^2 / (2 sigma_v^2)) on a grid padded by (K-1)/2
 * spaxels and (Kl-1)/2 channels, convolved with the K x K PSF in every
 * channel and the Kl-tap line-spread function along every spaxel (valid
 * part, as gf_convolve_psf and gf_line_model), plus a constant continuum.
 * Parameters per cube (GF_CUBE_NPAR, FP64):
 *   [xc, yc, Ie, Re, n, q, phi, continuum, v0, vproj, rt, sigma_v].
 * chi^2 = sum over voxels of w (d - m)^2.
 *
 * All cubes of a batch share Nc (1..GF_CUBE_MAX_CHAN) and the odd LSF length
 * Kl (1..GF_LINE_MAX_K); H, W and the odd PSF side K vary per cube (H + K - 1
 * and W + K - 1 at most GF_MAX_FFT).  Flat layouts: cube s's data, weight
 * and model occupy voxels [vox_off[s], vox_off[s+1]) (Nc H W each), its PSF
 * taps [psf_off[s], psf_off[s+1]), its LSF taps [lsf_off[s], lsf_off[s+1]),
 * its parameters [par_off[s], par_off[s+1]).  The batch owns the device
 * workspace its calls need (grown on first use). */
#define GF_CUBE_NPAR 12
#define GF_CUBE_MAX_CHAN 1024
typedef struct gf_cube_batch gf_cube_batch;

gf_status gf_cube_batch_create(gf_ctx *ctx, int n, const int32_t *H, const int32_t *W, const int32_t *K, int n_chan,
                               int K_lsf, gf_cube_batch **out);
void gf_cube_batch_destroy(gf_cube_batch *cb);
/* Host arrays of n + 1 offsets each (any may be NULL). */
gf_status gf_cube_batch_offsets(const gf_cube_batch *cb, int64_t *vox_off, int64_t *psf_off, int64_t *lsf_off,
                                int64_t *par_off);
/* Kernels of every cube: psf device [psf_off[n]], lsf device [lsf_off[n]]
 * (both copied into the batch); conv_mode as gf_psf_prepare for the spatial
 * convolution.  Must precede the calls below.  gf_cube_batch_destroy frees
 * the batch's device memory: call it once the work on it has finished. */
gf_status gf_cube_set_kernels(gf_ctx *ctx, gf_cube_batch *cb, const float *psf, const float *lsf, int conv_mode);
/* Steps 1-2 plus continuum: out (device [vox_off[n]]) = the model cubes.
 * theta: device [par_off[n]] FP64; oversample S 1..8, oversample_v Sv 1..8. */
gf_status gf_cube_model(gf_ctx *ctx, gf_cube_batch *cb, const double *theta, int oversample, int oversample_v,
                        float *out);
/* Steps 1-3: chi2 (device [2 n]) compensated (hi, lo) FP32 pairs as in
 * gf_chi2; data, weight: device [vox_off[n]]. */
gf_status gf_cube_chi2(gf_ctx *ctx, gf_cube_batch *cb, const double *theta, int oversample, int oversample_v,
                       const float *data, const float *weight, float *chi2);
/* d model / d theta: out (device [GF_CUBE_NPAR * vox_off[n]]); cube s holds
 * GF_CUBE_NPAR cubes of Nc H W values from GF_CUBE_NPAR * vox_off[s], in
 * parameter order (the continuum's all ones). */
gf_status gf_cube_jacobian(gf_ctx *ctx, gf_cube_batch *cb, const double *theta, int oversample, int oversample_v,
                           float *out);
/* Levenberg-Marquardt over every cube with the rule of gf_fit_lm (opts:
 * max_iter, oversample, lambda0/up/down/max, ftol, xtol, lo, hi, free_mask,
 * poll_every, start as there; use_graph and speculate are unused).
 * theta_io: device [par_off[n]] FP64; res: device [n]. */
gf_status gf_cube_fit_lm(gf_ctx *ctx, gf_cube_batch *cb, const float *data, const float *weight, double *theta_io,
                         const gf_lm_opts *opts, int oversample_v, gf_lm_result *res);

/* Library version string. */
const char *gf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */

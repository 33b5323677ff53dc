/*
 * gfo.c -- plain FP64 CPU oracle for the galaxy-fitting hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * What it computes (Barsdell, Barnes & Fluke, "Fitting Galaxies on GPUs",
 * Sec. 2, the five-step fitting loop; Sec. 3, steps 1-3 as transform, FFT and
 * reduce):
 *   step 1  model evaluation on the pixel grid     -> gfo_eval_padded
 *   step 2  convolution with the PSF               -> gfo_conv_valid (direct;
 *           the paper does this in Fourier space, which reaches the same
 *           linear convolution up to rounding, so the definition is used)
 *   step 3  comparison, sum of squared differences -> gfo_chi2
 *   step 4/5 parameter update and stop test        -> gfo_fit_lm
 *           (Levenberg-Marquardt, the routine the paper attributes to galfit)
 *
 * The paper names the steps but not the profile, the sub-pixel sampling, the
 * convolution boundary, the weights or the optimiser's constants.  The
 * readings taken here are:
 *   - profile: elliptical Sersic  I = Ie exp(-b_n [(R/Re)^(1/n) - 1]),
 *     R^2 = x'^2 + y'^2/q^2 with (x', y') the offsets rotated by the position
 *     angle phi (counter-clockwise from +x, radians); b_n is the root of
 *     P(2n, b_n) = 1/2 with P the regularised lower incomplete gamma.
 *   - pixel (row i, col j) is centred on (x=j, y=i); its value is the mean of
 *     S x S midpoint sub-samples at x = j + (s+1/2)/S - 1/2 (same in y).
 *   - the model is evaluated on a padded grid of (H+K-1) x (W+K-1) pixels,
 *     stamp pixels -c .. H-1+c with c = (K-1)/2, and the PSF convolution keeps
 *     the "valid" H x W part:  out[y][x] = sum_{u,v} P[u][v] Mp[y+K-1-u][x+K-1-v].
 *   - the sky is a constant added after the convolution.
 *   - chi^2 = sum_i w_i (d_i - m_i)^2 with w the supplied inverse variance.
 *   - parameters per component: [x0, y0, Ie, Re, n, q, phi]; then one sky.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NPC 7 /* parameters per component */

/* ------------------------------------------------------------------ threads */
void gfo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int gfo_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* --------------------------------------------- incomplete gamma and b_n ---- */
/*
 * Regularised lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a).
 * For x < a + 1 the power series
 *     gamma(a, x) = x^a e^-x  sum_{k>=0} x^k / (a (a+1) ... (a+k))
 * converges quickly; otherwise the upper function Q = 1 - P is taken from its
 * Legendre continued fraction
 *     Gamma(a, x) = x^a e^-x / (x + 1 - a - 1(1-a)/(x + 3 - a - 2(2-a)/(x + 5 - a - ...)))
 * evaluated with the modified Lentz method.
 */
double gfo_gammp(double a, double x) {
  if (!(a > 0.0)) return NAN;
  if (x <= 0.0) return 0.0;
  double lpre = a * log(x) - x - lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term, den = a;
    for (int k = 1; k < 100000; ++k) {
      den += 1.0;
      term *= x / den;
      sum += term;
      if (fabs(term) <= fabs(sum) * 1e-17) break;
    }
    return sum * exp(lpre);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a;
  double c = 1.0 / tiny;
  double d = 1.0 / b;
  double h = d;
  for (int i = 1; i < 100000; ++i) {
    double an = -(double)i * ((double)i - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    double del = d * c;
    h *= del;
    if (fabs(del - 1.0) <= 1e-17) break;
  }
  return 1.0 - exp(lpre) * h;
}

/* dP/dx = x^(a-1) e^-x / Gamma(a) */
double gfo_dgammp_dx(double a, double x) {
  if (x <= 0.0) return 0.0;
  return exp((a - 1.0) * log(x) - x - lgamma(a));
}

/*
 * b_n: the root of P(2n, b) = 1/2 (half the total light inside Re).  The
 * median of a gamma distribution lies below its mean, so the root is
 * bracketed by (0, 2n).  Start from the asymptotic value 2n - 1/3
 * (Ciotti & Bertin 1999) and refine by Newton steps, falling back to
 * bisection whenever a step leaves the bracket.
 */
double gfo_bn(double n) {
  if (!(n > 0.0)) return NAN;
  const double a = 2.0 * n;
  double lo = 0.0, hi = a;
  double b = a - 1.0 / 3.0;
  if (!(b > lo && b < hi)) b = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    double f = gfo_gammp(a, b) - 0.5;
    if (f > 0.0) hi = b; else lo = b;
    double fp = gfo_dgammp_dx(a, b);
    double nb = b - f / fp;
    if (!(nb > lo && nb < hi) || !isfinite(nb)) nb = 0.5 * (lo + hi);
    if (fabs(nb - b) <= 1e-16 * fabs(b) || hi - lo <= 1e-16 * fabs(b)) { b = nb; break; }
    b = nb;
  }
  return b;
}

/*
 * db_n/dn by implicit differentiation of P(2n, b_n) = 1/2:
 *     2 dP/da + dP/dx * b'_n = 0   =>   b'_n = -2 (dP/da) / (dP/dx),
 * with dP/da taken by an FP64 central difference.
 */
double gfo_dbn(double n) {
  const double a = 2.0 * n;
  const double b = gfo_bn(n);
  const double h = 1e-5 * a;
  double dpa = (gfo_gammp(a + h, b) - gfo_gammp(a - h, b)) / (2.0 * h);
  return -2.0 * dpa / gfo_dgammp_dx(a, b);
}

/* ------------------------------------------------------- Sersic component --- */
typedef struct {
  double x0, y0, ie, re, n, q, phi;
  double bn, dbn, cs, sn;
} comp_t;

static void load_comps(int ncomp, const double *theta, comp_t *c, int want_dbn) {
  for (int k = 0; k < ncomp; ++k) {
    const double *t = theta + NPC * k;
    c[k].x0 = t[0]; c[k].y0 = t[1]; c[k].ie = t[2]; c[k].re = t[3];
    c[k].n = t[4]; c[k].q = t[5]; c[k].phi = t[6];
    c[k].bn = gfo_bn(t[4]);
    c[k].dbn = want_dbn ? gfo_dbn(t[4]) : 0.0;
    c[k].cs = cos(t[6]);
    c[k].sn = sin(t[6]);
  }
}

/* Surface brightness of one component at the point (x, y). */
static double sersic_at(const comp_t *c, double x, double y) {
  double dx = x - c->x0, dy = y - c->y0;
  double xp = dx * c->cs + dy * c->sn;
  double yp = -dx * c->sn + dy * c->cs;
  double r = sqrt(xp * xp + yp * yp / (c->q * c->q));
  return c->ie * exp(-c->bn * (pow(r / c->re, 1.0 / c->n) - 1.0));
}

/*
 * Value and the seven partial derivatives d I / d[x0, y0, Ie, Re, n, q, phi]
 * of one component at (x, y).  With u = R/Re, t = u^(1/n), E = b_n t:
 *   dI/dIe = I/Ie,  dI/dRe = I E/(n Re),  dI/dn = I (b'_n (1-t) + E ln(u)/n^2),
 *   dI/d(R^2) = -I E/(2 n R^2) combined with the derivatives of
 *   R^2 = x'^2 + y'^2/q^2 with respect to x0, y0, q and phi.
 * At R = 0 exactly the value is Ie e^{b_n} and the terms that carry 1/R^2 or
 * ln u are taken as zero.
 */
static double sersic_grad_at(const comp_t *c, double x, double y, double *g) {
  double dx = x - c->x0, dy = y - c->y0;
  double xp = dx * c->cs + dy * c->sn;
  double yp = -dx * c->sn + dy * c->cs;
  double q2 = c->q * c->q;
  double r2 = xp * xp + yp * yp / q2;
  double n = c->n;
  if (r2 == 0.0) {
    double I = c->ie * exp(c->bn);
    g[0] = 0.0; g[1] = 0.0; g[2] = I / c->ie; g[3] = 0.0;
    g[4] = I * c->dbn; /* t = 0: dI/dn = I b'_n */
    g[5] = 0.0; g[6] = 0.0;
    return I;
  }
  double u = sqrt(r2) / c->re;
  double t = pow(u, 1.0 / n);
  double I = c->ie * exp(-c->bn * (t - 1.0));
  double E = c->bn * t;
  double dI_dr2 = -I * E / (2.0 * n * r2);
  double dr2_dx0 = -2.0 * xp * c->cs + 2.0 * yp * c->sn / q2;
  double dr2_dy0 = -2.0 * xp * c->sn - 2.0 * yp * c->cs / q2;
  double dr2_dq = -2.0 * yp * yp / (q2 * c->q);
  double dr2_dphi = 2.0 * xp * yp * (1.0 - 1.0 / q2);
  g[0] = dI_dr2 * dr2_dx0;
  g[1] = dI_dr2 * dr2_dy0;
  g[2] = I / c->ie;
  g[3] = I * E / (n * c->re);
  g[4] = I * (c->dbn * (1.0 - t) + E * log(u) / (n * n));
  g[5] = dI_dr2 * dr2_dq;
  g[6] = dI_dr2 * dr2_dphi;
  return I;
}

/* Pixel value (all components, no sky) at stamp pixel (i, j): the mean of the
 * S x S sub-samples.  (i, j) may lie in the padding (negative or >= size). */
static double pixel_value(int ncomp, const comp_t *c, int S, int i, int j) {
  double acc = 0.0;
  for (int sy = 0; sy < S; ++sy) {
    double y = (double)i + ((double)sy + 0.5) / (double)S - 0.5;
    for (int sx = 0; sx < S; ++sx) {
      double x = (double)j + ((double)sx + 0.5) / (double)S - 0.5;
      for (int k = 0; k < ncomp; ++k) acc += sersic_at(&c[k], x, y);
    }
  }
  return acc / ((double)S * (double)S);
}

static void pixel_grad(int ncomp, const comp_t *c, int S, int i, int j, double *out) {
  double g[NPC];
  for (int p = 0; p < NPC * ncomp; ++p) out[p] = 0.0;
  for (int sy = 0; sy < S; ++sy) {
    double y = (double)i + ((double)sy + 0.5) / (double)S - 0.5;
    for (int sx = 0; sx < S; ++sx) {
      double x = (double)j + ((double)sx + 0.5) / (double)S - 0.5;
      for (int k = 0; k < ncomp; ++k) {
        sersic_grad_at(&c[k], x, y, g);
        for (int p = 0; p < NPC; ++p) out[NPC * k + p] += g[p];
      }
    }
  }
  double inv = 1.0 / ((double)S * (double)S);
  for (int p = 0; p < NPC * ncomp; ++p) out[p] *= inv;
}

double gfo_sersic_point(const double *comp7, double x, double y) {
  comp_t c;
  load_comps(1, comp7, &c, 0);
  return sersic_at(&c, x, y);
}

double gfo_pixel(int ncomp, const double *theta, int S, int i, int j) {
  comp_t *c = (comp_t *)malloc(sizeof(comp_t) * (size_t)ncomp);
  load_comps(ncomp, theta, c, 0);
  double v = pixel_value(ncomp, c, S, i, j);
  free(c);
  return v;
}

/* Padded model grid (step 1): out has (H+K-1) rows of (W+K-1); padded index
 * (pi, pj) is stamp pixel (pi - c, pj - c). */
void gfo_eval_padded(int H, int W, int K, int ncomp, const double *theta, int S, double *out) {
  int c0 = (K - 1) / 2, Mh = H + K - 1, Mw = W + K - 1;
  comp_t *c = (comp_t *)malloc(sizeof(comp_t) * (size_t)ncomp);
  load_comps(ncomp, theta, c, 0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int pi = 0; pi < Mh; ++pi)
    for (int pj = 0; pj < Mw; ++pj)
      out[(size_t)pi * Mw + pj] = pixel_value(ncomp, c, S, pi - c0, pj - c0);
  free(c);
}

/* Same grid, each component into its own plane: out[k][Mh*Mw]. */
void gfo_eval_padded_comps(int H, int W, int K, int ncomp, const double *theta, int S, double *out) {
  int Mh = H + K - 1, Mw = W + K - 1;
  size_t plane = (size_t)Mh * Mw;
  for (int k = 0; k < ncomp; ++k)
    gfo_eval_padded(H, W, K, 1, theta + NPC * k, S, out + plane * k);
}

/* ------------------------------------------------------------ convolution --- */
double gfo_conv_valid_pixel(const double *mp, int Mh, int Mw, const double *psf, int K, int y, int x) {
  (void)Mh;
  double acc = 0.0;
  for (int u = 0; u < K; ++u)
    for (int v = 0; v < K; ++v)
      acc += psf[u * K + v] * mp[(size_t)(y + K - 1 - u) * Mw + (x + K - 1 - v)];
  return acc;
}

/* Step 2 as its definition: "valid" linear convolution of the padded grid. */
void gfo_conv_valid(const double *mp, int Mh, int Mw, const double *psf, int K, double *out) {
  int H = Mh - K + 1, W = Mw - K + 1;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      out[(size_t)y * W + x] = gfo_conv_valid_pixel(mp, Mh, Mw, psf, K, y, x);
}

/* Full model: convolved components plus the constant sky. */
void gfo_model(int H, int W, int K, int ncomp, const double *theta, int S, const double *psf, double *out) {
  int Mh = H + K - 1, Mw = W + K - 1;
  double *mp = (double *)malloc(sizeof(double) * (size_t)Mh * Mw);
  gfo_eval_padded(H, W, K, ncomp, theta, S, mp);
  gfo_conv_valid(mp, Mh, Mw, psf, K, out);
  double sky = theta[NPC * ncomp];
  for (size_t i = 0; i < (size_t)H * W; ++i) out[i] += sky;
  free(mp);
}

/* ------------------------------------------------------------------- chi^2 --- */
/* Step 3: chi^2 = sum w (d - m)^2; resid (nullable) = sqrt(w) (d - m). */
double gfo_chi2(long npix, const double *d, const double *w, const double *m, double *resid) {
  double acc = 0.0;
  for (long i = 0; i < npix; ++i) {
    double r = sqrt(w[i]) * (d[i] - m[i]);
    if (resid) resid[i] = r;
    acc += r * r;
  }
  return acc;
}

/* ---------------------------------------------------------------- Jacobian --- */
/*
 * Per-pixel derivative images of the model:  jac[p][H*W] = d m / d theta_p.
 * Each component derivative is the PSF convolution of the sub-sample mean of
 * the point derivative; d m / d sky = 1.
 */
void gfo_dpixel(int ncomp, const double *theta, int S, int i, int j, double *out) {
  comp_t *c = (comp_t *)malloc(sizeof(comp_t) * (size_t)ncomp);
  load_comps(ncomp, theta, c, 1);
  pixel_grad(ncomp, c, S, i, j, out);
  free(c);
}

void gfo_dpadded(int H, int W, int K, int ncomp, const double *theta, int S, double *out /*[7*ncomp][Mh*Mw]*/) {
  int c0 = (K - 1) / 2, Mh = H + K - 1, Mw = W + K - 1;
  size_t plane = (size_t)Mh * Mw;
  int np = NPC * ncomp;
  comp_t *c = (comp_t *)malloc(sizeof(comp_t) * (size_t)ncomp);
  load_comps(ncomp, theta, c, 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int pi = 0; pi < Mh; ++pi) {
    double g[NPC * 16];
    double *gp = np <= NPC * 16 ? g : (double *)malloc(sizeof(double) * (size_t)np);
    for (int pj = 0; pj < Mw; ++pj) {
      pixel_grad(ncomp, c, S, pi - c0, pj - c0, gp);
      for (int p = 0; p < np; ++p) out[plane * p + (size_t)pi * Mw + pj] = gp[p];
    }
    if (gp != g) free(gp);
  }
  free(c);
}

void gfo_jacobian(int H, int W, int K, int ncomp, const double *theta, int S, const double *psf, double *jac) {
  int Mh = H + K - 1, Mw = W + K - 1, np = NPC * ncomp;
  size_t plane = (size_t)Mh * Mw, npix = (size_t)H * W;
  double *dp = (double *)malloc(sizeof(double) * plane * (size_t)np);
  gfo_dpadded(H, W, K, ncomp, theta, S, dp);
  for (int p = 0; p < np; ++p) gfo_conv_valid(dp + plane * p, Mh, Mw, psf, K, jac + npix * p);
  for (size_t i = 0; i < npix; ++i) jac[npix * np + i] = 1.0;
  free(dp);
}

/* Gradient of chi^2:  d chi^2 / d theta_p = -2 sum_i w_i (d_i - m_i) d m_i / d theta_p. */
void gfo_grad_chi2(int H, int W, int K, int ncomp, const double *theta, int S, const double *psf,
                   const double *d, const double *w, double *grad) {
  int P = NPC * ncomp + 1;
  size_t npix = (size_t)H * W;
  double *m = (double *)malloc(sizeof(double) * npix);
  double *jac = (double *)malloc(sizeof(double) * npix * (size_t)P);
  gfo_model(H, W, K, ncomp, theta, S, psf, m);
  gfo_jacobian(H, W, K, ncomp, theta, S, psf, jac);
  for (int p = 0; p < P; ++p) {
    double acc = 0.0;
    for (size_t i = 0; i < npix; ++i) acc += w[i] * (d[i] - m[i]) * jac[npix * p + i];
    grad[p] = -2.0 * acc;
  }
  free(m);
  free(jac);
}

/* -------------------------------------------------------- Levenberg-Marquardt */
/* Cholesky factorisation of the n x n matrix a (row-major, overwritten by L). */
static int cholesky(int n, double *a) {
  for (int j = 0; j < n; ++j) {
    double s = a[j * n + j];
    for (int k = 0; k < j; ++k) s -= a[j * n + k] * a[j * n + k];
    if (!(s > 0.0) || !isfinite(s)) return -1;
    double ljj = sqrt(s);
    a[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = a[i * n + j];
      for (int k = 0; k < j; ++k) t -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = t / ljj;
    }
  }
  return 0;
}

static void chol_solve(int n, const double *l, const double *b, double *x) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= l[i * n + k] * x[k];
    x[i] = s / l[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * x[k];
    x[i] = s / l[i * n + i];
  }
}

/*
 * Levenberg-Marquardt (Marquardt 1963) over the free parameters:
 *   A = J^T W J, g = J^T W (d - m), D = diag(max(A_ii, 1e-12 max_j A_jj));
 *   solve (A + lambda D) delta = g by Cholesky (if A + lambda D is not positive
 *   definite: lambda *= up and retry);  theta' = clip(theta + delta, lo, hi).
 *   chi2' < chi2 (strictly): accept, lambda /= down, stop when
 *     (chi2 - chi2')/chi2' < ftol  or  max_i |delta_i| / max(|theta_i|, 1) < xtol;
 *   otherwise reject and lambda *= up; stop when lambda > lambda_max.
 *   A model that already fits exactly (chi2 = 0) stops at once.
 * dopt = {lambda0, lambda_up, lambda_down, lambda_max, ftol, xtol}.
 * res  = {chi2, lambda, iters, nfev, njev, status, reason} with status 0
 * (converged) or 6 (not converged) and reason 1 ftol, 2 xtol, 3 zero chi2,
 * 4 lambda above lambda_max, 5 iteration cap.
 * Returns 0, or -1 on invalid arguments.
 */
int gfo_fit_lm(int H, int W, int K, int ncomp, int S, const double *psf, const double *d, const double *w,
               const unsigned char *free_mask, const double *lo, const double *hi, int max_iter,
               const double *dopt, double *theta, double *res_d, int *res_i) {
  if (H <= 0 || W <= 0 || K <= 0 || (K % 2) == 0 || ncomp <= 0 || S <= 0) return -1;
  const int P = NPC * ncomp + 1;
  const size_t npix = (size_t)H * W;
  double lambda = dopt[0];
  const double up = dopt[1], down = dopt[2], lmax = dopt[3], ftol = dopt[4], xtol = dopt[5];

  int nf = 0, idx[64];
  for (int p = 0; p < P; ++p)
    if (!free_mask || free_mask[p]) idx[nf++] = p;

  double *m = (double *)malloc(sizeof(double) * npix);
  double *jac = (double *)malloc(sizeof(double) * npix * (size_t)P);
  double *A = (double *)calloc((size_t)nf * nf, sizeof(double));
  double *Ad = (double *)calloc((size_t)nf * nf, sizeof(double));
  double *g = (double *)calloc((size_t)nf, sizeof(double));
  double *delta = (double *)calloc((size_t)nf, sizeof(double));
  double *trial = (double *)malloc(sizeof(double) * P);

  for (int p = 0; p < P; ++p) {
    if (lo && theta[p] < lo[p]) theta[p] = lo[p];
    if (hi && theta[p] > hi[p]) theta[p] = hi[p];
  }
  gfo_model(H, W, K, ncomp, theta, S, psf, m);
  double chi2 = gfo_chi2((long)npix, d, w, m, NULL);
  int nfev = 1, njev = 0, status = 6, reason = 5, it = 0;
  int need_jac = 1;

  if (chi2 == 0.0) {
    status = 0;
    reason = 3;
  } else {
    for (it = 1; it <= max_iter; ++it) {
      if (need_jac) {
        gfo_jacobian(H, W, K, ncomp, theta, S, psf, jac);
        ++njev;
        for (int a = 0; a < nf; ++a) {
          const double *ja = jac + npix * idx[a];
          double s = 0.0;
          for (size_t i = 0; i < npix; ++i) s += ja[i] * w[i] * (d[i] - m[i]);
          g[a] = s;
          for (int b = 0; b <= a; ++b) {
            const double *jb = jac + npix * idx[b];
            double t = 0.0;
            for (size_t i = 0; i < npix; ++i) t += ja[i] * w[i] * jb[i];
            A[a * nf + b] = t;
            A[b * nf + a] = t;
          }
        }
        need_jac = 0;
      }
      double dmax = 0.0;
      for (int a = 0; a < nf; ++a)
        if (A[a * nf + a] > dmax) dmax = A[a * nf + a];
      memcpy(Ad, A, sizeof(double) * (size_t)nf * nf);
      for (int a = 0; a < nf; ++a) {
        double da = A[a * nf + a];
        if (da < 1e-12 * dmax) da = 1e-12 * dmax;
        Ad[a * nf + a] += lambda * da;
      }
      if (cholesky(nf, Ad) != 0) {
        lambda *= up;
        if (lambda > lmax) { status = 6; reason = 4; break; }
        continue;
      }
      chol_solve(nf, Ad, g, delta);
      memcpy(trial, theta, sizeof(double) * P);
      for (int a = 0; a < nf; ++a) {
        int p = idx[a];
        double v = theta[p] + delta[a];
        if (lo && v < lo[p]) v = lo[p];
        if (hi && v > hi[p]) v = hi[p];
        trial[p] = v;
      }
      double *mt = (double *)malloc(sizeof(double) * npix);
      gfo_model(H, W, K, ncomp, trial, S, psf, mt);
      double chi2t = gfo_chi2((long)npix, d, w, mt, NULL);
      ++nfev;
      if (chi2t < chi2) {
        double step = 0.0;
        for (int a = 0; a < nf; ++a) {
          int p = idx[a];
          double sc = fabs(theta[p]) > 1.0 ? fabs(theta[p]) : 1.0;
          double s = fabs(trial[p] - theta[p]) / sc;
          if (s > step) step = s;
        }
        double rel = chi2t > 0.0 ? (chi2 - chi2t) / chi2t : 0.0;
        memcpy(theta, trial, sizeof(double) * P);
        memcpy(m, mt, sizeof(double) * npix);
        free(mt);
        chi2 = chi2t;
        lambda /= down;
        need_jac = 1;
        if (chi2 == 0.0) { status = 0; reason = 3; break; }
        if (rel < ftol) { status = 0; reason = 1; break; }
        if (step < xtol) { status = 0; reason = 2; break; }
      } else {
        free(mt);
        lambda *= up;
        if (lambda > lmax) { status = 6; reason = 4; break; }
      }
    }
    if (it > max_iter) { it = max_iter; status = 6; reason = 5; }
  }

  res_d[0] = chi2;
  res_d[1] = lambda;
  res_i[0] = it;
  res_i[1] = nfev;
  res_i[2] = njev;
  res_i[3] = status;
  res_i[4] = reason;
  free(m); free(jac); free(A); free(Ad); free(g); free(delta); free(trial);
  return 0;
}

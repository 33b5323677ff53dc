// cnn_api.cpp -- host side of the learned starting-point proposal: the
// network object (FP32 master weights, BF16 mirrors, Adam moments and the
// activation workspace for one batch), its forward, gradient and training
// entry points, the parameter coding, and the on-device random numbers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gf_internal.h"

namespace gf {
hipError_t launch_gemm(hipStream_t, bool, bool, const bf16_t *, int, const bf16_t *, int, int, int, int, const Epi &,
                       float *, int64_t);
hipError_t launch_border_stats(hipStream_t, const float *, int, int, int, float2 *);
hipError_t launch_im2col_first(hipStream_t, const float *, const float2 *, int, int, bf16_t *);
hipError_t launch_im2col(hipStream_t, const bf16_t *, int, int, int, bf16_t *);
hipError_t launch_col2im_relu(hipStream_t, const float *, const bf16_t *, int, int, int, bf16_t *);
hipError_t launch_colsum(hipStream_t, const void *, bool, int, int, float *, float *);
int colsum_chunks(int M);
hipError_t launch_mse(hipStream_t, const float *, const float *, int, float *, bf16_t *, float *);
hipError_t launch_adam(hipStream_t, int64_t, float *, const float *, float *, float *, bf16_t *, float, float, float,
                       float, float, float);
hipError_t launch_to_bf16(hipStream_t, int64_t, const float *, bf16_t *);
hipError_t launch_encode(hipStream_t, int, int, const float *, float *);
hipError_t launch_decode(hipStream_t, int, int, const float *, double *);
hipError_t launch_philox_raw(hipStream_t, uint64_t, uint64_t, const uint64_t *, int64_t, uint64_t *);
hipError_t launch_normal_noise(hipStream_t, uint64_t, uint64_t, const uint64_t *, int64_t, float, const float *,
                               float *);
hipError_t launch_draw_prior(hipStream_t, uint64_t, uint64_t, const uint64_t *, int, int, float *);
hipError_t launch_init_uniform(hipStream_t, uint64_t, uint64_t, const uint64_t *, int64_t, float, float *);
hipError_t launch_moments(hipStream_t, const gf_batch *, const float *, int, double *);
}  // namespace gf

using namespace gf;

namespace {

constexpr int kConvC[5] = {1, 32, 32, 64, 64};
constexpr int kFc1 = 256, kOut = 8, kBorder = 4;
constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

gf_status cfail(gf_ctx *c, gf_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

#define CNN_TRY(ctx, expr)                                                                                   \
  do {                                                                                                       \
    hipError_t e_ = (expr);                                                                                  \
    if (e_ != hipSuccess) return cfail(ctx, GF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One parameter tensor: canonical [rows][cols] and its place in the internal
// flat layout, where the first-layer weights are padded from 9 to 16 columns.
struct Tensor {
  int rows, cols, icols;
  int64_t coff, ioff;
  float lim;      // He-uniform bound sqrt(6/fan_in); 0 for biases
};

}  // namespace

struct gf_cnn {
  gf_ctx *ctx = nullptr;
  int side = 0, mb = 0;
  std::vector<Tensor> t;    // w1 b1 w2 b2 w3 b3 w4 b4 w5 b5 w6 b6
  int64_t n_canon = 0, n_int = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  bf16_t *pb = nullptr;
  int64_t step = 0;
  // activations and workspace for mb stamps
  float2 *stats = nullptr;
  bf16_t *col[4] = {};      // im2col of layers 1..4
  bf16_t *act[5] = {};      // act[1..4]: layer outputs (act[4] is the flattened dense input)
  bf16_t *h = nullptr, *dyb = nullptr, *dh = nullptr;
  bf16_t *dz[5] = {};       // dz[1..4]: gradients at the layer outputs after the ReLU derivative
  float *y = nullptr, *dy = nullptr, *dcol = nullptr, *part = nullptr, *cpart = nullptr, *loss = nullptr;
  int64_t part_cap = 0;
  char *mem = nullptr;
};

namespace {

int side_at(const gf_cnn *n, int layer) { return n->side >> layer; }   // output side of conv layer `layer` (1..4)

void dfree_any(void *p) {
  if (p) (void)hipFree(p);
}

struct Bump {
  char *base = nullptr;
  size_t off = 0;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~(size_t)255;
    T *r = base ? (T *)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    return r;
  }
};

void layout(gf_cnn *n, Bump &b) {
  const int64_t mb = n->mb;
  n->p = b.take<float>(n->n_int);
  n->g = b.take<float>(n->n_int);
  n->m = b.take<float>(n->n_int);
  n->v = b.take<float>(n->n_int);
  n->pb = b.take<bf16_t>(n->n_int);
  n->stats = b.take<float2>(mb);
  int64_t maxdcol = 0;
  for (int l = 1; l <= 4; ++l) {
    const int64_t rows = mb * side_at(n, l) * side_at(n, l);
    const int kcols = l == 1 ? 16 : 9 * kConvC[l - 1];
    n->col[l - 1] = b.take<bf16_t>(rows * kcols);
    n->act[l] = b.take<bf16_t>(rows * kConvC[l]);
    n->dz[l] = b.take<bf16_t>(rows * kConvC[l]);
    if (l > 1) maxdcol = std::max(maxdcol, rows * kcols);
  }
  n->h = b.take<bf16_t>(mb * kFc1);
  n->dh = b.take<bf16_t>(mb * kFc1);
  n->y = b.take<float>(mb * kOut);
  n->dy = b.take<float>(mb * kOut);
  n->dyb = b.take<bf16_t>(mb * kOut);
  n->dcol = b.take<float>(maxdcol);
  n->part_cap = 8ll << 20;
  n->part = b.take<float>(n->part_cap);
  n->cpart = b.take<float>((int64_t)colsum_chunks((int)(mb * side_at(n, 1) * side_at(n, 1))) * kFc1);
  n->loss = b.take<float>(1);
}

hipError_t gemm(gf_cnn *n, bool ak, bool bk, const bf16_t *A, int lda, const bf16_t *B, int ldb, int M, int N, int K,
                const Epi &e) {
  return launch_gemm(n->ctx->stream, ak, bk, A, lda, B, ldb, M, N, K, e, n->part, n->part_cap);
}

Epi epi_none() { return Epi{nullptr, 0, nullptr, 0, nullptr, 0, nullptr, 0}; }

// Forward pass of nb stamps at x (device [nb][side][side]); logits in n->y.
gf_status forward(gf_cnn *n, const float *x, int nb) {
  gf_ctx *c = n->ctx;
  hipStream_t st = c->stream;
  CNN_TRY(c, launch_border_stats(st, x, nb, n->side, kBorder, n->stats));
  CNN_TRY(c, launch_im2col_first(st, x, n->stats, nb, n->side, n->col[0]));
  for (int l = 1; l <= 4; ++l) {
    const int so = side_at(n, l);
    const int M = nb * so * so, N = kConvC[l], K = n->t[2 * (l - 1)].icols;
    if (l > 1) CNN_TRY(c, launch_im2col(st, n->act[l - 1], nb, side_at(n, l - 1), kConvC[l - 1], n->col[l - 1]));
    Epi e = epi_none();
    e.bias = n->p + n->t[2 * (l - 1) + 1].ioff;
    e.relu = 1;
    e.outb = n->act[l];
    e.ldb = N;
    CNN_TRY(c, gemm(n, true, true, n->col[l - 1], K, n->pb + n->t[2 * (l - 1)].ioff, K, M, N, K, e));
  }
  const int F = n->t[8].cols;
  Epi e5 = epi_none();
  e5.bias = n->p + n->t[9].ioff;
  e5.relu = 1;
  e5.outb = n->h;
  e5.ldb = kFc1;
  CNN_TRY(c, gemm(n, true, true, n->act[4], F, n->pb + n->t[8].ioff, F, nb, kFc1, F, e5));
  Epi e6 = epi_none();
  e6.bias = n->p + n->t[11].ioff;
  e6.outf = n->y;
  e6.ldf = kOut;
  CNN_TRY(c, gemm(n, true, true, n->h, kFc1, n->pb + n->t[10].ioff, kFc1, nb, kOut, kFc1, e6));
  return GF_OK;
}

// Gradients of the mean squared error against targets into n->g (after forward).
gf_status backward(gf_cnn *n, const float *targets, int nb) {
  gf_ctx *c = n->ctx;
  hipStream_t st = c->stream;
  const int F = n->t[8].cols;
  CNN_TRY(c, launch_mse(st, n->y, targets, nb * kOut, n->dy, n->dyb, n->loss));
  // dense 2
  Epi e = epi_none();
  e.outf = n->g + n->t[10].ioff;
  e.ldf = kFc1;
  CNN_TRY(c, gemm(n, false, false, n->dyb, kOut, n->h, kFc1, kOut, kFc1, nb, e));
  CNN_TRY(c, launch_colsum(st, n->dy, false, nb, kOut, n->cpart, n->g + n->t[11].ioff));
  e = epi_none();
  e.mask = n->h;
  e.ldm = kFc1;
  e.outb = n->dh;
  e.ldb = kFc1;
  CNN_TRY(c, gemm(n, true, false, n->dyb, kOut, n->pb + n->t[10].ioff, kFc1, nb, kFc1, kOut, e));
  // dense 1
  e = epi_none();
  e.outf = n->g + n->t[8].ioff;
  e.ldf = F;
  CNN_TRY(c, gemm(n, false, false, n->dh, kFc1, n->act[4], F, kFc1, F, nb, e));
  CNN_TRY(c, launch_colsum(st, n->dh, true, nb, kFc1, n->cpart, n->g + n->t[9].ioff));
  e = epi_none();
  e.mask = n->act[4];
  e.ldm = F;
  e.outb = n->dz[4];
  e.ldb = F;
  CNN_TRY(c, gemm(n, true, false, n->dh, kFc1, n->pb + n->t[8].ioff, F, nb, F, kFc1, e));
  // convolutions 4..1
  for (int l = 4; l >= 1; --l) {
    const int so = side_at(n, l);
    const int M = nb * so * so, Co = kConvC[l], Kc = n->t[2 * (l - 1)].icols;
    e = epi_none();
    e.outf = n->g + n->t[2 * (l - 1)].ioff;
    e.ldf = Kc;
    CNN_TRY(c, gemm(n, false, false, n->dz[l], Co, n->col[l - 1], Kc, Co, Kc, M, e));
    CNN_TRY(c, launch_colsum(st, n->dz[l], true, M, Co, n->cpart, n->g + n->t[2 * (l - 1) + 1].ioff));
    if (l == 1) break;
    e = epi_none();
    e.outf = n->dcol;
    e.ldf = Kc;
    CNN_TRY(c, gemm(n, true, false, n->dz[l], Co, n->pb + n->t[2 * (l - 1)].ioff, Kc, M, Kc, Co, e));
    CNN_TRY(c, launch_col2im_relu(st, n->dcol, n->act[l - 1], nb, side_at(n, l - 1), kConvC[l - 1], n->dz[l - 1]));
  }
  return GF_OK;
}

gf_status check_batch(gf_cnn *n, const void *x, int nb, const char *who) {
  if (!n || !x) return cfail(n ? n->ctx : nullptr, GF_EINVAL, std::string(who) + ": null argument");
  if (nb <= 0 || nb > n->mb)
    return cfail(n->ctx, GF_ESHAPE, std::string(who) + ": batch of " + std::to_string(nb) + " outside 1.." +
                                        std::to_string(n->mb));
  return GF_OK;
}

}  // namespace

extern "C" {

gf_status gf_cnn_create(gf_ctx *c, int side, int max_batch, gf_cnn **out) {
  if (!c || !out) return cfail(c, GF_EINVAL, "gf_cnn_create: null argument");
  *out = nullptr;
  if (side < 16 || side % 16 != 0 || side > 1024) return cfail(c, GF_ESHAPE, "gf_cnn_create: side must be 16..1024, a multiple of 16");
  if (max_batch <= 0 || (int64_t)max_batch * side * side > (1ll << 31))
    return cfail(c, GF_ESHAPE, "gf_cnn_create: max_batch * side^2 must be positive and at most 2^31");
  gf_cnn *n = new (std::nothrow) gf_cnn();
  if (!n) return GF_ENOMEM;
  n->ctx = c;
  n->side = side;
  n->mb = max_batch;
  const int F = (side / 16) * (side / 16) * kConvC[4];
  const int shp[6][2] = {{32, 9}, {32, 288}, {64, 288}, {64, 576}, {kFc1, F}, {kOut, kFc1}};
  int64_t co = 0, io = 0;
  for (int l = 0; l < 6; ++l) {
    const int r = shp[l][0], cc = shp[l][1], ic = l == 0 ? 16 : cc;
    n->t.push_back(Tensor{r, cc, ic, co, io, (float)std::sqrt(6.0 / cc)});
    co += (int64_t)r * cc;
    io += ((int64_t)r * ic + 63) / 64 * 64;
    n->t.push_back(Tensor{1, r, r, co, io, 0.f});
    co += r;
    io += (r + 63) / 64 * 64;
  }
  n->n_canon = co;
  n->n_int = io;
  Bump b;
  layout(n, b);
  if (hipMalloc((void **)&n->mem, b.off) != hipSuccess) {
    delete n;
    return cfail(c, GF_ENOMEM, "gf_cnn_create: allocation of " + std::to_string(b.off) + " bytes failed");
  }
  b.base = n->mem;
  b.off = 0;
  layout(n, b);
  if (hipMemsetAsync(n->p, 0, 5 * n->n_int * sizeof(float), c->stream) != hipSuccess ||
      hipMemsetAsync(n->pb, 0, n->n_int * sizeof(bf16_t), c->stream) != hipSuccess) {
    dfree_any(n->mem);
    delete n;
    return cfail(c, GF_EDEVICE, "gf_cnn_create: clearing parameters failed");
  }
  *out = n;
  return GF_OK;
}

void gf_cnn_destroy(gf_cnn *n) {
  if (!n) return;
  // hipFree waits for the device; the context may already be gone.
  dfree_any(n->mem);
  delete n;
}

int64_t gf_cnn_param_count(const gf_cnn *n) { return n ? n->n_canon : 0; }

static gf_status reset_adam(gf_cnn *n) {
  gf_ctx *c = n->ctx;
  n->step = 0;
  CNN_TRY(c, hipMemsetAsync(n->m, 0, n->n_int * sizeof(float), c->stream));
  CNN_TRY(c, hipMemsetAsync(n->v, 0, n->n_int * sizeof(float), c->stream));
  CNN_TRY(c, launch_to_bf16(c->stream, n->n_int, n->p, n->pb));
  return GF_OK;
}

gf_status gf_cnn_init(gf_cnn *n, uint64_t key) {
  if (!n) return GF_EINVAL;
  gf_ctx *c = n->ctx;
  ProfBind pb(c);
  CNN_TRY(c, hipMemsetAsync(n->p, 0, n->n_int * sizeof(float), c->stream));
  for (size_t i = 0; i < n->t.size(); i += 2) {
    const Tensor &w = n->t[i];
    const uint64_t ctr[4] = {0, (uint64_t)i / 2, 0, 0};
    CNN_TRY(c, hipMemsetAsync(n->p + w.ioff, 0, (size_t)w.rows * w.icols * sizeof(float), c->stream));
    // draw rows x cols values, then place them into the (possibly padded) rows
    float *dst = n->p + w.ioff;
    if (w.icols == w.cols) {
      CNN_TRY(c, launch_init_uniform(c->stream, key, 0x5eed, ctr, (int64_t)w.rows * w.cols, w.lim, dst));
    } else {
      float *tmp = n->g;   // gradients are scratch until the next backward pass
      CNN_TRY(c, launch_init_uniform(c->stream, key, 0x5eed, ctr, (int64_t)w.rows * w.cols, w.lim, tmp));
      CNN_TRY(c, hipMemcpy2DAsync(dst, w.icols * sizeof(float), tmp, w.cols * sizeof(float), w.cols * sizeof(float),
                                  w.rows, hipMemcpyDeviceToDevice, c->stream));
    }
  }
  CNN_TRY(c, hipMemsetAsync(n->g, 0, n->n_int * sizeof(float), c->stream));
  return reset_adam(n);
}

gf_status gf_cnn_set_params(gf_cnn *n, const float *params) {
  if (!n || !params) return cfail(n ? n->ctx : nullptr, GF_EINVAL, "gf_cnn_set_params: null argument");
  gf_ctx *c = n->ctx;
  CNN_TRY(c, hipMemsetAsync(n->p, 0, n->n_int * sizeof(float), c->stream));
  for (const Tensor &w : n->t)
    CNN_TRY(c, hipMemcpy2DAsync(n->p + w.ioff, w.icols * sizeof(float), params + w.coff, w.cols * sizeof(float),
                                w.cols * sizeof(float), w.rows, hipMemcpyDeviceToDevice, c->stream));
  return reset_adam(n);
}

static gf_status get_canon(gf_cnn *n, const float *src, float *out) {
  gf_ctx *c = n->ctx;
  for (const Tensor &w : n->t)
    CNN_TRY(c, hipMemcpy2DAsync(out + w.coff, w.cols * sizeof(float), src + w.ioff, w.icols * sizeof(float),
                                w.cols * sizeof(float), w.rows, hipMemcpyDeviceToDevice, c->stream));
  return GF_OK;
}

gf_status gf_cnn_get_params(gf_cnn *n, float *out) {
  if (!n || !out) return cfail(n ? n->ctx : nullptr, GF_EINVAL, "gf_cnn_get_params: null argument");
  return get_canon(n, n->p, out);
}

gf_status gf_cnn_forward(gf_cnn *n, const float *stamps, int count, float *out) {
  if (!n || !stamps || !out || count < 0) return cfail(n ? n->ctx : nullptr, GF_EINVAL, "gf_cnn_forward: bad argument");
  gf_ctx *c = n->ctx;
  ProfBind pb(c);
  const int64_t px = (int64_t)n->side * n->side;
  for (int s0 = 0; s0 < count; s0 += n->mb) {
    const int nb = std::min(n->mb, count - s0);
    gf_status r = forward(n, stamps + s0 * px, nb);
    if (r != GF_OK) return r;
    CNN_TRY(c, hipMemcpyAsync(out + (int64_t)s0 * kOut, n->y, (size_t)nb * kOut * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
  }
  return GF_OK;
}

gf_status gf_cnn_gradients(gf_cnn *n, const float *stamps, const float *targets, int count, float *grads,
                           float *loss) {
  gf_status r = check_batch(n, stamps, count, "gf_cnn_gradients");
  if (r != GF_OK) return r;
  if (!targets) return cfail(n->ctx, GF_EINVAL, "gf_cnn_gradients: null targets");
  gf_ctx *c = n->ctx;
  ProfBind pb(c);
  if ((r = forward(n, stamps, count)) != GF_OK) return r;
  if ((r = backward(n, targets, count)) != GF_OK) return r;
  if (grads && (r = get_canon(n, n->g, grads)) != GF_OK) return r;
  if (loss) CNN_TRY(c, hipMemcpyAsync(loss, n->loss, sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  return GF_OK;
}

gf_status gf_cnn_train_step(gf_cnn *n, const float *stamps, const float *targets, int count, float lr, float *loss) {
  gf_status r = gf_cnn_gradients(n, stamps, targets, count, nullptr, loss);
  if (r != GF_OK) return r;
  gf_ctx *c = n->ctx;
  ProfBind pb(c);
  n->step += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)kAdamB1, (double)n->step));
  const double c2 = 1.0 / (1.0 - std::pow((double)kAdamB2, (double)n->step));
  CNN_TRY(c, launch_adam(c->stream, n->n_int, n->p, n->g, n->m, n->v, n->pb, lr, kAdamB1, kAdamB2, kAdamEps,
                         (float)c1, (float)c2));
  return GF_OK;
}

int64_t gf_cnn_steps(const gf_cnn *n) { return n ? n->step : 0; }

gf_status gf_cnn_encode(gf_ctx *c, int count, int side, const float *theta, float *targets) {
  if (!c || count < 0 || (count > 0 && (!theta || !targets)) || side < 16)
    return cfail(c, GF_EINVAL, "gf_cnn_encode: bad argument");
  CNN_TRY(c, launch_encode(c->stream, count, side, theta, targets));
  return GF_OK;
}

gf_status gf_cnn_decode(gf_ctx *c, int count, int side, const float *targets, double *theta) {
  if (!c || count < 0 || (count > 0 && (!theta || !targets)) || side < 16)
    return cfail(c, GF_EINVAL, "gf_cnn_decode: bad argument");
  ProfBind pb(c);
  CNN_TRY(c, launch_decode(c->stream, count, side, targets, theta));
  return GF_OK;
}

gf_status gf_philox(gf_ctx *c, uint64_t key0, uint64_t key1, const uint64_t *counter, int64_t n_blocks,
                    uint64_t *out) {
  if (!c || n_blocks < 0 || (n_blocks > 0 && !out)) return cfail(c, GF_EINVAL, "gf_philox: bad argument");
  CNN_TRY(c, launch_philox_raw(c->stream, key0, key1, counter, n_blocks, out));
  return GF_OK;
}

gf_status gf_normal_noise(gf_ctx *c, int64_t n, float sigma, uint64_t key0, uint64_t key1, const uint64_t *counter,
                          const float *clean, float *out) {
  if (!c || n < 0 || (n > 0 && !out)) return cfail(c, GF_EINVAL, "gf_normal_noise: bad argument");
  ProfBind pb(c);
  CNN_TRY(c, launch_normal_noise(c->stream, key0, key1, counter, n, sigma, clean, out));
  return GF_OK;
}

gf_status gf_draw_prior(gf_ctx *c, int count, int side, uint64_t key0, uint64_t key1, const uint64_t *counter,
                        float *theta) {
  if (!c || count < 0 || (count > 0 && !theta) || side < 16) return cfail(c, GF_EINVAL, "gf_draw_prior: bad argument");
  ProfBind pb(c);
  CNN_TRY(c, launch_draw_prior(c->stream, key0, key1, counter, count, side, theta));
  return GF_OK;
}

gf_status gf_moments_guess(gf_ctx *c, const gf_batch *b, const float *data, double *theta) {
  if (!c || !b || !data || !theta) return cfail(c, GF_EINVAL, "gf_moments_guess: null argument");
  int p2 = 1;
  for (const StampDesc &d : b->h_desc) {
    if (d.ncomp != 1) return cfail(c, GF_ESHAPE, "gf_moments_guess: every stamp must have one component");
    if (d.H < 9 || d.W < 9) return cfail(c, GF_ESHAPE, "gf_moments_guess: stamps must be at least 9 x 9");
    const int nf = d.H * d.W - (d.H - 8) * (d.W - 8);
    if (nf > 16384) return cfail(c, GF_ESHAPE, "gf_moments_guess: outer frame above 16384 pixels");
    while (p2 < nf) p2 <<= 1;
  }
  ProfBind pb(c);
  CNN_TRY(c, launch_moments(c->stream, b, data, p2, theta));
  return GF_OK;
}

}  // extern "C"

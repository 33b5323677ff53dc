// tune.cpp -- the context's tuning table: which FFT form the automatic path
// choice takes per one-workgroup side (measured on the device the first
// time a side is used, when the context was created with a tuning file),
// and per bucket of those sides the fewest still-fitting stamps for which
// an LM fit keeps that form (set by the caller or read from the file).  The
// table is kept in that file as JSON keyed by the GPU architecture and
// name, so later contexts take the same choices (and hence give the same
// bits) without measuring again.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gf_internal.h"

using namespace gf;

namespace {

std::string device_key(int device, std::string *name) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  if (name) *name = prop.name;
  return arch;
}

// Reads `"key": {"<int>": <int>, ...}` pairs from a JSON object body.
void read_int_map(const std::string &txt, const char *key, std::vector<std::pair<int, int>> &out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = txt.find(k);
  if (p == std::string::npos) return;
  p = txt.find('{', p);
  const size_t e = txt.find('}', p);
  if (p == std::string::npos || e == std::string::npos) return;
  const std::string body = txt.substr(p + 1, e - p - 1);
  size_t i = 0;
  while (true) {
    const size_t q0 = body.find('"', i);
    if (q0 == std::string::npos) break;
    const size_t q1 = body.find('"', q0 + 1);
    const size_t colon = body.find(':', q1);
    if (q1 == std::string::npos || colon == std::string::npos) break;
    const int a = std::atoi(body.substr(q0 + 1, q1 - q0 - 1).c_str());
    const int b = std::atoi(body.c_str() + colon + 1);
    out.push_back({a, b});
    i = colon + 1;
  }
}

std::string read_string(const std::string &txt, const char *key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = txt.find(k);
  if (p == std::string::npos) return "";
  p = txt.find('"', txt.find(':', p));
  const size_t e = txt.find('"', p + 1);
  if (p == std::string::npos || e == std::string::npos) return "";
  return txt.substr(p + 1, e - p - 1);
}

// Median of `reps` timings (after one untimed run) of fn on the context's stream.
template <typename F>
gf_status time_us(gf_ctx *c, int reps, F fn, double *us) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return GF_EDEVICE;
  gf_status st = fn();
  std::vector<double> t;
  for (int r = 0; st == GF_OK && r < reps; ++r) {
    if (hipEventRecord(a, c->stream) != hipSuccess) st = GF_EDEVICE;
    if (st == GF_OK) st = fn();
    if (st == GF_OK && hipEventRecord(b, c->stream) != hipSuccess) st = GF_EDEVICE;
    float ms = 0.f;
    if (st == GF_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
      st = GF_EDEVICE;
    t.push_back(ms * 1e3);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != GF_OK) return st;
  std::sort(t.begin(), t.end());
  *us = t[t.size() / 2];
  return GF_OK;
}

// Time of a seven-channel convolution (one Jacobian's) of n H x H stamps
// with K x K PSFs in the given mode.
gf_status time_conv(gf_ctx *c, int H, int K, int n, int mode, double *us) {
  const int M = H + K - 1;
  std::vector<int32_t> hv(n, H), kv(n, K), nc(n, 1);
  gf_batch *b = nullptr;
  gf_status st = gf_batch_create(c, n, hv.data(), hv.data(), kv.data(), nc.data(), 0, &b);
  if (st != GF_OK) return st;
  float *taps = nullptr, *in = nullptr, *out = nullptr;
  const size_t n_taps = (size_t)n * K * K, n_in = (size_t)n * 7 * M * M, n_out = (size_t)n * 7 * H * H;
  gf_psf *p = nullptr;
  if (hipMalloc(&taps, n_taps * sizeof(float)) != hipSuccess || hipMalloc(&in, n_in * sizeof(float)) != hipSuccess ||
      hipMalloc(&out, n_out * sizeof(float)) != hipSuccess) {
    st = GF_ENOMEM;
  }
  // any finite values time the same: zeros for the input, a delta PSF
  if (st == GF_OK && (hipMemsetAsync(taps, 0, n_taps * sizeof(float), c->stream) != hipSuccess ||
                      hipMemsetAsync(in, 0, n_in * sizeof(float), c->stream) != hipSuccess))
    st = GF_EDEVICE;
  if (st == GF_OK) st = gf_psf_prepare(c, b, taps, mode, &p);
  if (st == GF_OK) st = time_us(c, 3, [&]() { return gf_convolve_psf(c, b, p, in, 7, out); }, us);
  if (hipStreamSynchronize(c->stream) != hipSuccess && st == GF_OK) st = GF_EDEVICE;
  gf_psf_destroy(p);
  gf_batch_destroy(b);
  if (taps) (void)hipFree(taps);
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  return st;
}

// The same for padded side L in the given FFT form.
gf_status time_form(gf_ctx *c, int L, int n, int mode, double *us) {
  const int K = L >= 24 ? 15 : 3;
  return time_conv(c, L - K + 1, K, n, mode, us);
}

}  // namespace

namespace gf {

gf_status tune_load(gf_ctx *c) {
  std::ifstream f(c->tune_path);
  if (!f) return GF_OK;   // no table yet: it is written on first tuning
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  std::string name;
  const std::string arch = device_key(c->device, &name);
  if (read_string(txt, "arch") != arch || read_string(txt, "device") != name) return GF_OK;   // another GPU
  std::vector<std::pair<int, int>> form, mina;
  read_int_map(txt, "form", form);
  read_int_map(txt, "min_active", mina);
  {
    const size_t k = txt.find("\"direct_max_k\"");
    if (k != std::string::npos) {
      const size_t colon = txt.find(':', k);
      const int v = colon == std::string::npos ? 0 : std::atoi(txt.c_str() + colon + 1);
      if (v >= 1 && v <= GF_MAX_K && (v % 2) == 1) {
        c->tune_direct_k = v;
        c->tune_direct_done = 1;
      }
    }
  }
  for (auto &kv : form) {
    const int k = f2d_class(kv.first);
    if (k >= 0 && (kv.second == 1 || kv.second == 2)) c->tune_form[k] = (int8_t)kv.second;
  }
  for (auto &kv : mina) {
    const int k = f2d_class(kv.first);
    if (k >= 0 && kv.second >= 0) {
      c->f2d_min_active[f2d_bucket(k)] = kv.second;
      c->tune_min_done[f2d_bucket(k)] = 1;
    }
  }
  return GF_OK;
}

gf_status tune_save(gf_ctx *c) {
  if (c->tune_path.empty()) return GF_OK;
  std::string name;
  const std::string arch = device_key(c->device, &name);
  std::ostringstream o;
  o << "{\"library\": \"" << gf_version() << "\", \"arch\": \"" << arch << "\", \"device\": \"" << name << "\",\n";
  if (c->tune_direct_done) o << " \"direct_max_k\": " << c->tune_direct_k << ",\n";
  o << " \"form\": {";
  bool first = true;
  for (int k = 0; k < kF2dN; ++k) {
    if (c->tune_form[k] < 0) continue;
    o << (first ? "" : ", ") << "\"" << kF2dSides[k] << "\": " << (int)c->tune_form[k];
    first = false;
  }
  o << "},\n \"min_active\": {";
  first = true;
  for (int b = 0; b < kF2dBuckets; ++b) {
    if (!c->tune_min_done[b]) continue;
    o << (first ? "" : ", ") << "\"" << kF2dSides[kF2dBucketEnd[b] - 1] << "\": " << c->f2d_min_active[b];
    first = false;
  }
  o << "}}\n";
  const std::string tmp = c->tune_path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return GF_EINVAL;
    f << o.str();
    if (!f) return GF_EINVAL;
  }
  if (std::rename(tmp.c_str(), c->tune_path.c_str()) != 0) return GF_EINVAL;
  return GF_OK;
}

// Measure the form of side L: 256 stamps of that padded side, one
// Jacobian's seven channels, the faster form kept.  (The switch threshold
// min_active is not measured here: convolutions of a few stamps of one side
// favour the one-workgroup form, but in a fit's last iterations the few
// remaining stamps of every bucket run one launch per bucket, where the
// multi-pass form covers all sides in three; the default rule, eight rounds
// of workgroups, was the fastest on the uneven batch.)
gf_status tune_side(gf_ctx *c, int L) {
  const int k = f2d_class(L);
  if (k < 0) return GF_OK;
  double tf = 0, tm = 0;
  gf_status st = time_form(c, L, 256, GF_CONV_FFT_FUSED, &tf);
  if (st == GF_OK) st = time_form(c, L, 256, GF_CONV_FFT_MULTIPASS, &tm);
  if (st != GF_OK) return st;
  c->tune_form[k] = (int8_t)(tf <= tm ? 2 : 1);
  // a table that cannot be written (a read-only place) is only not kept
  (void)tune_save(c);
  return GF_OK;
}

// The direct-path threshold: 256 stamps of 64 x 64 in seven channels, each
// odd K from 3 to 15 convolved directly and by FFT; the threshold is the
// largest K up to which the direct path is not slower (the direct cost grows
// as K^2, the FFT's barely with K, so the first K where the FFT wins ends
// the scan).
gf_status tune_direct(gf_ctx *c) {
  int best = 1;
  for (int K = 3; K <= 15; K += 2) {
    double td = 0, tf = 0;
    gf_status st = time_conv(c, 64, K, 256, GF_CONV_DIRECT, &td);
    if (st == GF_OK) st = time_conv(c, 64, K, 256, GF_CONV_FFT, &tf);
    if (st != GF_OK) return st;
    if (td > tf) break;
    best = K;
  }
  c->tune_direct_k = best;
  c->tune_direct_done = 1;
  (void)tune_save(c);
  return GF_OK;
}

}  // namespace gf

extern "C" gf_status gf_autotune(gf_ctx *c, const int32_t *sides, int n_sides) {
  if (!c || n_sides < 0 || (n_sides > 0 && !sides)) return GF_EINVAL;
  std::vector<int> todo;
  if (n_sides == 0) {
    for (int k = 0; k < kF2dN; ++k) todo.push_back(kF2dSides[k]);
  } else {
    for (int i = 0; i < n_sides; ++i) {
      if (f2d_class(sides[i]) < 0) {
        c->err = "gf_autotune: " + std::to_string(sides[i]) + " is not a one-workgroup FFT side";
        return GF_EINVAL;
      }
      todo.push_back(sides[i]);
    }
  }
  for (int L : todo) {
    gf_status st = tune_side(c, L);
    if (st != GF_OK) {
      if (c->err.empty()) c->err = "gf_autotune: measuring side " + std::to_string(L) + " failed";
      return st;
    }
  }
  if (n_sides == 0) {
    gf_status st = tune_direct(c);
    if (st != GF_OK) {
      if (c->err.empty()) c->err = "gf_autotune: measuring the direct-path threshold failed";
      return st;
    }
  }
  return GF_OK;
}

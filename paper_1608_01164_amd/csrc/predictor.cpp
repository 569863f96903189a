// C ABI of the rank predictor: creation, parameters, forward, loss gradient, Adam training, and
// training rows from recorded solves.
#include "predictor.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hq.h"
#include "engine.h"

hq_predictor_s::~hq_predictor_s() {
  for (float* p : {d_params, d_m, d_v, d_grad, d_part})
    if (p) (void)hipFree(p);
}

namespace hq {

void predictor_features(float* x, int64_t n, int b, int l, int64_t block, int k, double a_k, double c_k,
                        double r_prev, double l0, double tol) {
  x[0] = (float)(l / 8.0);
  x[1] = (float)(std::log2((double)std::max<int64_t>(block, 1)) / 16.0);
  x[2] = (float)(std::log2(b + 1.0) / 4.0);
  x[3] = (float)(k / 8.0);
  x[4] = (float)(std::log10(std::max(c_k, 1.0)) / 12.0);
  x[5] = (float)(std::log10(std::max(a_k, 1.0)) / 6.0);
  x[6] = rank_code(r_prev);
  x[7] = (float)(std::log10(1.0 / std::max(l0, 1e-300)) / 16.0);
  x[8] = (float)(std::log2((double)std::max<int64_t>(n, 1)) / 20.0);
  x[9] = (float)(std::log10(1.0 / tol) / 16.0);
}

int predictor_capacity(float code, float margin, int64_t cmax) {
  const double c = std::min(std::max((double)code + margin, 0.0), 1.2);  // rank <= 2^12
  const int64_t cap = (int64_t)std::ceil(std::exp2(10.0 * c) - 1.0) + 4;
  return (int)std::max<int64_t>(1, std::min(cap, cmax));
}

}  // namespace hq

namespace {

hq_status pfail(hq_status s, const char* m) {
  hq::set_last_error(m);
  return s;
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool ok(hipError_t e) { return e == hipSuccess; }

bool ensure_part(hq_predictor_s* p, int64_t rows) {
  const int64_t g = hq::mlp_groups(rows);
  if (g <= p->part_groups) return true;
  if (p->d_part) (void)hipFree(p->d_part);
  p->d_part = nullptr;
  p->part_groups = 0;
  if (!ok(hipMalloc(&p->d_part, sizeof(float) * (size_t)g * (hq::kMlpParams + 1)))) return false;
  p->part_groups = g;
  return true;
}

bool weight_sum(const float* W, int64_t rows, hipStream_t st, double& sum) {
  std::vector<float> w((size_t)rows * hq::kMlpOutputs);
  if (!ok(hipMemcpyAsync(w.data(), W, sizeof(float) * w.size(), hipMemcpyDeviceToHost, st))) return false;
  if (!ok(hipStreamSynchronize(st))) return false;
  sum = 0.0;
  for (float v : w) sum += v;
  return true;
}

}  // namespace

extern "C" {

int64_t hq_predictor_nparams(void) { return hq::kMlpParams; }

hq_status hq_predictor_create(uint64_t seed, hq_predictor_t* out) {
  if (!out) return pfail(HQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  hq_predictor_s* p = new hq_predictor_s();
  const size_t P = hq::kMlpParams;
  if (!ok(hipMalloc(&p->d_params, sizeof(float) * P)) || !ok(hipMalloc(&p->d_m, sizeof(float) * P)) ||
      !ok(hipMalloc(&p->d_v, sizeof(float) * P)) || !ok(hipMalloc(&p->d_grad, sizeof(float) * (P + 1)))) {
    delete p;
    return pfail(HQ_ERR_ALLOC, "predictor allocation failed");
  }
  // Glorot-uniform weights, zero biases
  constexpr int F = hq::kMlpFeatures, H = hq::kMlpHidden, O = hq::kMlpOutputs;
  std::vector<float> w(P, 0.0f);
  uint64_t s = seed;
  auto fill = [&](size_t off, int fan_out, int fan_in) {
    const double lim = std::sqrt(6.0 / (fan_in + fan_out));
    for (int i = 0; i < fan_out * fan_in; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * 0x1.0p-53;  // [0, 1)
      w[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  fill(0, H, F);
  fill(H * F + H, H, H);
  fill(H * F + H + H * H + H, O, H);
  std::vector<float> z(P, 0.0f);
  if (!ok(hipMemcpy(p->d_params, w.data(), sizeof(float) * P, hipMemcpyHostToDevice)) ||
      !ok(hipMemcpy(p->d_m, z.data(), sizeof(float) * P, hipMemcpyHostToDevice)) ||
      !ok(hipMemcpy(p->d_v, z.data(), sizeof(float) * P, hipMemcpyHostToDevice))) {
    delete p;
    return pfail(HQ_ERR_DEVICE, "predictor upload failed");
  }
  *out = p;
  return HQ_OK;
}

hq_status hq_predictor_get_params(hq_predictor_t p, float* params) {
  if (!p || !params) return pfail(HQ_ERR_ARG, "NULL argument");
  if (!ok(hipMemcpy(params, p->d_params, sizeof(float) * hq::kMlpParams, hipMemcpyDeviceToHost)))
    return pfail(HQ_ERR_DEVICE, "parameter download failed");
  return HQ_OK;
}

hq_status hq_predictor_set_params(hq_predictor_t p, const float* params) {
  if (!p || !params) return pfail(HQ_ERR_ARG, "NULL argument");
  if (!ok(hipMemcpy(p->d_params, params, sizeof(float) * hq::kMlpParams, hipMemcpyHostToDevice)))
    return pfail(HQ_ERR_DEVICE, "parameter upload failed");
  return HQ_OK;
}

hq_status hq_predictor_set_margin(hq_predictor_t p, const float* margin) {
  if (!p || !margin) return pfail(HQ_ERR_ARG, "NULL argument");
  for (int o = 0; o < hq::kMlpOutputs; ++o) {
    if (!(margin[o] >= 0.0f && margin[o] <= 1.0f)) return pfail(HQ_ERR_ARG, "margin outside [0, 1]");
    p->margin[o] = margin[o];
  }
  return HQ_OK;
}

hq_status hq_predictor_get_margin(hq_predictor_t p, float* margin) {
  if (!p || !margin) return pfail(HQ_ERR_ARG, "NULL argument");
  for (int o = 0; o < hq::kMlpOutputs; ++o) margin[o] = p->margin[o];
  return HQ_OK;
}

hq_status hq_predictor_forward(hq_predictor_t p, const float* X, int64_t rows, float* Y, void* stream) {
  if (!p || rows < 0) return pfail(HQ_ERR_ARG, "bad arguments");
  if (rows == 0) return HQ_OK;
  if (!X || !Y) return pfail(HQ_ERR_ARG, "X or Y is NULL");
  try {
    hq::launch_mlp_forward(p->d_params, X, nullptr, Y, rows, (hipStream_t)stream);
  } catch (const std::exception& e) {
    return pfail(HQ_ERR_DEVICE, e.what());
  }
  return HQ_OK;
}

hq_status hq_predictor_loss_grad(hq_predictor_t p, const float* X, const float* T, const float* W, int64_t rows,
                                 float* loss, float* grad, void* stream) {
  if (!p || !X || !T || !W || !loss || !grad || rows < 1) return pfail(HQ_ERR_ARG, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  double wsum = 0.0;
  if (!weight_sum(W, rows, st, wsum)) return pfail(HQ_ERR_DEVICE, "weight readback failed");
  if (!(wsum > 0.0)) return pfail(HQ_ERR_ARG, "all weights are zero");
  if (!ensure_part(p, rows)) return pfail(HQ_ERR_ALLOC, "workspace allocation failed");
  try {
    hq::launch_mlp_grad(p->d_params, X, T, W, rows, (float)(1.0 / wsum), p->d_part, p->d_grad, st);
  } catch (const std::exception& e) {
    return pfail(HQ_ERR_DEVICE, e.what());
  }
  if (!ok(hipMemcpyAsync(grad, p->d_grad, sizeof(float) * hq::kMlpParams, hipMemcpyDeviceToDevice, st)) ||
      !ok(hipMemcpyAsync(loss, p->d_grad + hq::kMlpParams, sizeof(float), hipMemcpyDeviceToHost, st)) ||
      !ok(hipStreamSynchronize(st)))
    return pfail(HQ_ERR_DEVICE, "gradient failed");
  return HQ_OK;
}

hq_status hq_predictor_train(hq_predictor_t p, const float* X, const float* T, const float* W, int64_t rows,
                             int32_t epochs, float lr, void* stream, float* loss) {
  if (!p || !X || !T || !W || rows < 1 || epochs < 1 || !(lr > 0.0f)) return pfail(HQ_ERR_ARG, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  double wsum = 0.0;
  if (!weight_sum(W, rows, st, wsum)) return pfail(HQ_ERR_DEVICE, "weight readback failed");
  if (!(wsum > 0.0)) return pfail(HQ_ERR_ARG, "all weights are zero");
  if (!ensure_part(p, rows)) return pfail(HQ_ERR_ALLOC, "workspace allocation failed");
  try {
    for (int e = 0; e < epochs; ++e) {
      hq::launch_mlp_grad(p->d_params, X, T, W, rows, (float)(1.0 / wsum), p->d_part, p->d_grad, st);
      hq::launch_mlp_adam(p->d_params, p->d_m, p->d_v, p->d_grad, lr, (int)(++p->step), st);
    }
  } catch (const std::exception& ex) {
    (void)hipStreamSynchronize(st);
    return pfail(HQ_ERR_DEVICE, ex.what());
  }
  float l = 0.0f;
  if (!ok(hipMemcpyAsync(&l, p->d_grad + hq::kMlpParams, sizeof(float), hipMemcpyDeviceToHost, st)) ||
      !ok(hipStreamSynchronize(st)))
    return pfail(HQ_ERR_DEVICE, "training failed");
  if (loss) *loss = l;
  return HQ_OK;
}

hq_status hq_predictor_rows(const hq_info* info, int64_t n, int32_t b, const hq_opts* opts, float* X, float* T,
                            float* W, int32_t* rows) {
  if (!info || !opts || !X || !T || !W || !rows || n < 1 || b < 1) return pfail(HQ_ERR_ARG, "bad arguments");
  hq::Tree t;
  t.build(n, opts->leaf);
  if (t.L > 24 || info->iters > 16) return pfail(HQ_ERR_UNSUPPORTED, "more than 24 levels or 16 iterations");
  const int beff = (int)std::min<int64_t>(b, std::max<int64_t>(1, n - 1));
  int r = 0;
  for (int k = 0; k < info->iters; ++k)
    for (int l = 0; l < t.L; ++l) {
      const double prev = k == 0 ? beff : info->level_ranks[k - 1][0][l];
      hq::predictor_features(X + (size_t)r * hq::kMlpFeatures, n, beff, l, t.ldf[l], k, info->a[k], info->c[k], prev,
                             info->l0, opts->tol);
      for (int o = 0; o < hq::kMlpOutputs; ++o) {
        T[(size_t)r * hq::kMlpOutputs + o] = hq::rank_code(info->level_ranks[k][o][l]);
        W[(size_t)r * hq::kMlpOutputs + o] = (o == 0 || k >= 1) ? 1.0f : 0.0f;
      }
      ++r;
    }
  *rows = r;
  return HQ_OK;
}

void hq_predictor_destroy(hq_predictor_t p) { delete p; }

}  // extern "C"

// Rank predictor network: a fully connected F -> H -> H -> O perceptron with tanh hidden units
// and a linear output, in FP32.  Hand-written forward, backward (per-row backpropagation with
// per-workgroup partial gradients, summed in a fixed order) and Adam kernels.
//
// Parameter layout (flat, row-major): W1 (H x F), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O).
// Loss: sum_{i,o} w_io (y_io - t_io)^2 / sum w  (weighted squared error, w = 0 masks an entry).
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "mlp.h"

namespace hq {

namespace {
void check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("predictor kernel launch failed: ") + hipGetErrorString(e));
}

constexpr int F = kMlpFeatures, H = kMlpHidden, O = kMlpOutputs, P = kMlpParams;
constexpr int kW1 = 0, kB1 = kW1 + H * F, kW2 = kB1 + H, kB2 = kW2 + H * H, kW3 = kB2 + H, kB3 = kW3 + O * H;
static_assert(kB3 + O == P, "parameter layout");
constexpr int kRowsPerGroup = 128;  // rows of one workgroup in the gradient kernel (one thread each)

__device__ __forceinline__ void forward_row(const float* __restrict__ w, const float* x, float* h1, float* h2,
                                            float* y) {
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = w[kB1 + j];
#pragma unroll
    for (int f = 0; f < F; ++f) z += w[kW1 + j * F + f] * x[f];
    h1[j] = tanhf(z);
  }
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = w[kB2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) z += w[kW2 + j * H + i] * h1[i];
    h2[j] = tanhf(z);
  }
#pragma unroll
  for (int o = 0; o < O; ++o) {
    float z = w[kB3 + o];
#pragma unroll
    for (int j = 0; j < H; ++j) z += w[kW3 + o * H + j] * h2[j];
    y[o] = z;
  }
}
}  // namespace

// Y = net(X) for `rows` rows (row-major, F and O floats).  With prev != null, feature
// kMlpPrevFeature of row i is replaced by output 0 of row i of prev (the previous iteration's
// predicted rank code: features and targets share the encoding).
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     const float* __restrict__ prev, float* __restrict__ Y,
                                                     int64_t rows) {
  __shared__ float w[P];
  for (int i = threadIdx.x; i < P; i += 256) w[i] = params[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float x[F], h1[H], h2[H], y[O];
#pragma unroll
  for (int f = 0; f < F; ++f) x[f] = X[r * F + f];
  if (prev) x[kMlpPrevFeature] = prev[r * O + 0];
  forward_row(w, x, h1, h2, y);
#pragma unroll
  for (int o = 0; o < O; ++o) Y[r * O + o] = y[o];
}

// Partial gradients of the loss (scaled by inv_wsum) over kRowsPerGroup rows per workgroup:
// part[g * (P + 1) + p] for p < P, and the partial loss at index P.
__global__ __launch_bounds__(kRowsPerGroup) void k_mlp_grad(const float* __restrict__ params,
                                                            const float* __restrict__ X,
                                                            const float* __restrict__ T,
                                                            const float* __restrict__ Wt, int64_t rows,
                                                            float inv_wsum, float* __restrict__ part) {
  __shared__ float w[P];
  __shared__ float sx[kRowsPerGroup][F + 1];
  __shared__ float sh1[kRowsPerGroup][H + 1];
  __shared__ float sh2[kRowsPerGroup][H + 1];
  __shared__ float sd1[kRowsPerGroup][H + 1];  // dL/dz1
  __shared__ float sd2[kRowsPerGroup][H + 1];  // dL/dz2
  __shared__ float sd3[kRowsPerGroup][O + 1];  // dL/dy
  __shared__ float sl[kRowsPerGroup];
  const int tid = threadIdx.x;
  for (int i = tid; i < P; i += kRowsPerGroup) w[i] = params[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * kRowsPerGroup + tid;
  float x[F], h1[H], h2[H], y[O];
  if (r < rows) {
#pragma unroll
    for (int f = 0; f < F; ++f) x[f] = X[r * F + f];
    forward_row(w, x, h1, h2, y);
    float loss = 0.0f, d3[O];
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const float e = y[o] - T[r * O + o], wt = Wt[r * O + o];
      loss += wt * e * e;
      d3[o] = 2.0f * wt * e * inv_wsum;
    }
    sl[tid] = loss * inv_wsum;
    float d2[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      float g = 0.0f;
#pragma unroll
      for (int o = 0; o < O; ++o) g += w[kW3 + o * H + j] * d3[o];
      d2[j] = g * (1.0f - h2[j] * h2[j]);
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
      float g = 0.0f;
#pragma unroll
      for (int j = 0; j < H; ++j) g += w[kW2 + j * H + i] * d2[j];
      sd1[tid][i] = g * (1.0f - h1[i] * h1[i]);
    }
#pragma unroll
    for (int f = 0; f < F; ++f) sx[tid][f] = x[f];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      sh1[tid][j] = h1[j];
      sh2[tid][j] = h2[j];
      sd2[tid][j] = d2[j];
    }
#pragma unroll
    for (int o = 0; o < O; ++o) sd3[tid][o] = d3[o];
  } else {  // rows past the end contribute nothing
    sl[tid] = 0.0f;
#pragma unroll
    for (int f = 0; f < F; ++f) sx[tid][f] = 0.0f;
    for (int j = 0; j < H; ++j) {
      sh1[tid][j] = 0.0f;
      sh2[tid][j] = 0.0f;
      sd1[tid][j] = 0.0f;
      sd2[tid][j] = 0.0f;
    }
#pragma unroll
    for (int o = 0; o < O; ++o) sd3[tid][o] = 0.0f;
  }
  __syncthreads();
  // parameter p: sum over the group's rows of (upstream delta) x (input activation), fixed order
  float* out = part + (size_t)blockIdx.x * (P + 1);
  for (int p = tid; p < P; p += kRowsPerGroup) {
    float g = 0.0f;
    if (p < kB1) {
      const int j = (p - kW1) / F, f = (p - kW1) % F;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd1[q][j] * sx[q][f];
    } else if (p < kW2) {
      const int j = p - kB1;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd1[q][j];
    } else if (p < kB2) {
      const int j = (p - kW2) / H, i = (p - kW2) % H;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd2[q][j] * sh1[q][i];
    } else if (p < kW3) {
      const int j = p - kB2;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd2[q][j];
    } else if (p < kB3) {
      const int o = (p - kW3) / H, j = (p - kW3) % H;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd3[q][o] * sh2[q][j];
    } else {
      const int o = p - kB3;
      for (int q = 0; q < kRowsPerGroup; ++q) g += sd3[q][o];
    }
    out[p] = g;
  }
  if (tid == 0) {
    float l = 0.0f;
    for (int q = 0; q < kRowsPerGroup; ++q) l += sl[q];
    out[P] = l;
  }
}

// grad[p] = sum_g part[g][p] (and the loss at index P), in group order.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int groups,
                                                    float* __restrict__ grad) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > P) return;
  float g = 0.0f;
  for (int q = 0; q < groups; ++q) g += part[(size_t)q * (P + 1) + p];
  grad[p] = g;
}

// One Adam step (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ params, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ grad, float lr,
                                                  float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  constexpr float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

void launch_mlp_forward(const float* params, const float* X, const float* prev, float* Y, int64_t rows, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, params, X, prev, Y, rows);
  check_launch();
}

int mlp_groups(int64_t rows) { return (int)((rows + kRowsPerGroup - 1) / kRowsPerGroup); }

void launch_mlp_grad(const float* params, const float* X, const float* T, const float* W, int64_t rows, float inv_wsum,
                     float* part, float* grad, hipStream_t s) {
  const int g = mlp_groups(rows);
  if (g <= 0) return;
  hipLaunchKernelGGL(k_mlp_grad, dim3(g), dim3(kRowsPerGroup), 0, s, params, X, T, W, rows, inv_wsum, part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((P + 1 + 255) / 256), dim3(256), 0, s, part, g, grad);
  check_launch();
}

void launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((P + 255) / 256), dim3(256), 0, s, params, m, v, grad, lr, c1, c2);
  check_launch();
}

}  // namespace hq

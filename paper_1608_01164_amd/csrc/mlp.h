// Rank predictor network (see mlp.hip): sizes, feature encoding and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace hq {

constexpr int kMlpFeatures = 10;
constexpr int kMlpHidden = 32;
constexpr int kMlpOutputs = 4;  // rank codes of X_{k+1}, Z_k, L_k^{-1}, Y_k at one level
constexpr int kMlpParams = kMlpHidden * kMlpFeatures + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOutputs * kMlpHidden + kMlpOutputs;
constexpr int kMlpPrevFeature = 6;  // rank code of X_k at the same level

// Rank code: log2(1 + rank) / 10 (targets, and the previous-rank feature).
inline float rank_code(double r) { return (float)(std::log2(1.0 + r) / 10.0); }

void launch_mlp_forward(const float* params, const float* X, const float* prev, float* Y, int64_t rows, hipStream_t s);
int mlp_groups(int64_t rows);
// part: mlp_groups(rows) * (kMlpParams + 1) floats; grad: kMlpParams + 1 floats (loss last)
void launch_mlp_grad(const float* params, const float* X, const float* T, const float* W, int64_t rows, float inv_wsum,
                     float* part, float* grad, hipStream_t s);
void launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, int step, hipStream_t s);

}  // namespace hq

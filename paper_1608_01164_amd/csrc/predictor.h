// Rank predictor: device state of the network and the feature encoding shared by training rows
// and the solver's inference.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "mlp.h"

struct hq_predictor_s {
  float* d_params = nullptr;  // kMlpParams
  float* d_m = nullptr;       // Adam moments
  float* d_v = nullptr;
  float* d_grad = nullptr;    // kMlpParams + 1 (loss last)
  float* d_part = nullptr;    // per-workgroup partial gradients
  int64_t part_groups = 0;
  int64_t step = 0;           // Adam steps taken
  float margin[hq::kMlpOutputs] = {0.05f, 0.05f, 0.05f, 0.05f};  // added to predicted codes for capacities
  ~hq_predictor_s();
};

namespace hq {

// Feature row (kMlpFeatures floats) for level l (block size `block`) of iteration k of a problem
// of order n and bandwidth b, with weights (a_k, c_k), previous rank r_prev of X_k at that level,
// certified l0 and truncation tolerance tol.
void predictor_features(float* x, int64_t n, int b, int l, int64_t block, int k, double a_k, double c_k,
                        double r_prev, double l0, double tol);
// Capacity for a predicted rank code plus its margin: 2^(10 (y + margin)) - 1 + 4, in [1, cmax].
int predictor_capacity(float code, float margin, int64_t cmax);
// Message returned by hq_last_error() for the calling thread.
void set_last_error(const std::string& m);

}  // namespace hq

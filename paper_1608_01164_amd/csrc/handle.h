// The object behind hq_hodlr_t: a HODLR matrix on the device with the engine (arenas, descriptor
// staging, streams) that owns its memory.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>

#include "engine.h"
#include "hmatrix.h"

struct hq_hodlr_s {
  hq::Tree t;
  std::unique_ptr<hq::Engine> e;
  hq::HMat H;
  int* d_w = nullptr;     // device int: width of the current apply
  hipEvent_t done = nullptr;
  ~hq_hodlr_s() {
    if (done) (void)hipEventDestroy(done);
    e.reset();
  }
};

// Pinned descriptor memory that one product of the handle's matrix with a thin dense block needs
// (one task per leaf and two per off-diagonal block, plus the width fill), reserved when the handle
// is made so that applying the matrix later takes no new pinned memory.
inline void reserve_apply_staging(hq_hodlr_s& h) {
  const size_t tasks = (size_t)h.t.nleaves + 4 * (size_t)h.t.ninternal + 16;
  h.e->stage.reserve(tasks * sizeof(hq::GemmTask) + (size_t(64) << 10));
}

// The object behind hq_hmatrix_t: an H-matrix made from a HODLR one (whose leaves it shares).
struct hq_hmatrix_s {
  hq::HMatrixH H;
  int64_t hodlr_bytes = 0;  // storage of the source HODLR matrix with its actual ranks
};

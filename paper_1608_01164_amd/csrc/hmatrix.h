// H-matrix format with the standard admissibility condition (Sec. 3.1.2), built from a HODLR matrix.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

#include "engine.h"

namespace hq {

// min(diam t, diam s) <= dist(t, s) for the index intervals t = [t0, t1), s = [s0, s1) (eq. stand_adm).
bool h_admissible(int64_t t0, int64_t t1, int64_t s0, int64_t s1);

struct HMatrixH {
  struct LowRank {          // rows [r0, r0 + m) x cols [c0, c0 + n): U V^T, rank on the device
    int64_t r0, c0, m, n;
    double* U;
    double* V;
    int ld, cap;
    int* rank;
  };
  struct Dense {            // rows [r0, r0 + m) x cols [c0, c0 + n), column-major
    int64_t r0, c0, m, n;
    double* D;              // corner blocks (null for a HODLR leaf, read from `leaves`)
    int leaf;               // HODLR leaf index of a diagonal block
    bool from_leaf;
  };
  int64_t n = 0;
  std::unique_ptr<Engine> e;  // owns the blocks' device memory
  std::vector<LowRank> lr;
  std::vector<Dense> dn;
  std::vector<int> ranks;     // host copy of the low-rank blocks' ranks
  const double* leaves = nullptr;  // the source HODLR's leaves (diagonal blocks), borrowed
  int ldl = 0;
  int64_t bytes = 0;          // storage with the actual ranks: (m + n) rank per low-rank block, m n per dense one
  int max_rank = 0;
  // Partition, recompress the admissible sub-blocks at tol, form the dense corners (stream `st`,
  // synchronised on return).  The source must outlive this object (its leaves are borrowed).
  void convert(const HMat& src, double tol, hipStream_t st);
};

}  // namespace hq

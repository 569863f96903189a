// Cluster tree of the HODLR format (Sec. 3.1.1): host-only, so that the host parts of the library
// (the structured QR sweep, the Zolotarev coefficients) also build without the device compiler.
#include <algorithm>

#include "engine.h"

namespace hq {

void Tree::build(int64_t n_, int leaf_) {
  n = n_;
  leaf = leaf_;
  L = 0;
  while (((n + (int64_t(1) << L) - 1) >> L) > leaf) ++L;
  nnodes = (2 << L) - 1;
  ninternal = (1 << L) - 1;
  nleaves = 1 << L;
  lo.assign(nnodes, 0);
  hi.assign(nnodes, 0);
  hi[0] = n;
  for (int p = 0; p < ninternal; ++p) {
    const int64_t m = mid(p);
    lo[2 * p + 1] = lo[p];
    hi[2 * p + 1] = m;
    lo[2 * p + 2] = m;
    hi[2 * p + 2] = hi[p];
  }
  maxleaf = 0;
  for (int p = ninternal; p < nnodes; ++p) maxleaf = std::max(maxleaf, size(p));
  ldf.assign(L, 0);
  for (int l = 0; l < L; ++l) ldf[l] = (n + (int64_t(2) << l) - 1) >> (l + 1);
}

}  // namespace hq

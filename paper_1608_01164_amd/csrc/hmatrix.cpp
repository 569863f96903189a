// HODLR -> H-matrix conversion with the standard admissibility condition (Sec. 3.1.2, eq.
// stand_adm): the format the paper compares HODLR with in Example hodlrvshmatrix / Table
// storage_spec.  The partition reuses the HODLR cluster tree; a block t x s of two clusters on one
// level is admissible when min(diam t, diam s) <= dist(t, s), and the recursion over children pairs
// stops at an admissible block (low rank) or at a leaf cluster (dense).  Each HODLR off-diagonal
// block U V^T thereby splits into admissible sub-blocks U(rows) V(cols)^T, recompressed on their own
// at the truncation tolerance (their ranks are often lower than the parent's), and one dense corner
// next to the diagonal; the HODLR leaves stay the dense diagonal blocks.
#include "hmatrix.h"

#include <algorithm>
#include <stdexcept>

namespace hq {

bool h_admissible(int64_t t0, int64_t t1, int64_t s0, int64_t s1) {
  const int64_t diam = std::min(t1 - t0 - 1, s1 - s0 - 1);
  int64_t dist = 0;
  if (t1 <= s0)
    dist = s0 - t1 + 1;
  else if (s1 <= t0)
    dist = t0 - s1 + 1;
  return diam <= dist;
}

void HMatrixH::convert(const HMat& src, double tol, hipStream_t st) {
  const Tree& tr = *src.t;
  n = tr.n;
  e.reset(new Engine(st));
  e->tol = tol;
  lr.clear();
  dn.clear();
  // the partition: HODLR leaves are the dense diagonal blocks; every off-diagonal block (p, s) of
  // HODLR is the pair (rows, cols) = (a, b) or (b, a) of p's children, split recursively
  struct Item { int blk_p, blk_s; int rn, cn; };  // HODLR block, current row and column clusters
  std::vector<Item> work;
  for (int q = tr.ninternal; q < tr.nnodes; ++q) {
    Dense d{};
    d.r0 = d.c0 = tr.lo[q];
    d.m = d.n = tr.size(q);
    d.leaf = tr.leaf_index(q);
    d.from_leaf = true;
    dn.push_back(d);
  }
  for (int p = 0; p < tr.ninternal; ++p)
    for (int s = 0; s < 2; ++s) work.push_back(Item{p, s, s == 0 ? 2 * p + 1 : 2 * p + 2, s == 0 ? 2 * p + 2 : 2 * p + 1});
  std::vector<Item> lr_items, dn_items;
  while (!work.empty()) {
    const Item it = work.back();
    work.pop_back();
    const int64_t t0 = tr.lo[it.rn], t1 = tr.hi[it.rn], s0 = tr.lo[it.cn], s1 = tr.hi[it.cn];
    if (t1 <= t0 || s1 <= s0) continue;
    if (h_admissible(t0, t1, s0, s1))
      lr_items.push_back(it);
    else if (tr.is_leaf(it.rn) || tr.is_leaf(it.cn))
      dn_items.push_back(it);
    else
      for (int a = 1; a <= 2; ++a)
        for (int b = 1; b <= 2; ++b) work.push_back(Item{it.blk_p, it.blk_s, 2 * it.rn + a, 2 * it.cn + b});
  }
  // device storage: every low-rank block keeps its parent's capacity; dense corners their size
  std::vector<Engine::RecTask> rec;
  std::vector<GemmTask> gm;
  int maxm = 1, maxn = 1;
  for (const Item& it : lr_items) {
    const int p = it.blk_p, s = it.blk_s, l = Tree::level(p), ld = (int)tr.ldf[l];
    // rows of the block (p, s) start at the first row cluster's lo, columns likewise
    const int64_t R0 = tr.lo[s == 0 ? 2 * p + 1 : 2 * p + 2], C0 = tr.lo[s == 0 ? 2 * p + 2 : 2 * p + 1];
    LowRank b{};
    b.r0 = tr.lo[it.rn];
    b.c0 = tr.lo[it.cn];
    b.m = tr.size(it.rn);
    b.n = tr.size(it.cn);
    b.cap = std::max(1, src.cap[l]);
    b.ld = (int)std::max<int64_t>(b.m, b.n);
    b.U = e->persist.get<double>((size_t)b.ld * b.cap);
    b.V = e->persist.get<double>((size_t)b.ld * b.cap);
    b.rank = e->persist.get<int>(1);
    lr.push_back(b);
    Engine::RecTask r{};
    r.Us = src.U(p, s) + (b.r0 - R0);
    r.ldus = ld;
    r.m = (int)b.m;
    r.Vs = src.V(p, s) + (b.c0 - C0);
    r.ldvs = ld;
    r.n = (int)b.n;
    r.r = src.rk(p, s);
    r.rcap = b.cap;
    r.U = b.U;
    r.V = b.V;
    r.ldu = r.ldv = b.ld;
    r.rank = b.rank;
    r.kcap = b.cap;
    r.thresh = tol;
    r.fidx = 0;
    rec.push_back(r);
  }
  for (const Item& it : dn_items) {
    const int p = it.blk_p, s = it.blk_s, l = Tree::level(p), ld = (int)tr.ldf[l];
    const int64_t R0 = tr.lo[s == 0 ? 2 * p + 1 : 2 * p + 2], C0 = tr.lo[s == 0 ? 2 * p + 2 : 2 * p + 1];
    Dense d{};
    d.r0 = tr.lo[it.rn];
    d.c0 = tr.lo[it.cn];
    d.m = tr.size(it.rn);
    d.n = tr.size(it.cn);
    d.D = e->persist.get<double>((size_t)d.m * d.n);
    dn.push_back(d);
    GemmTask g{};  // D = U(rows) V(cols)^T over the parent's live rank
    g.A = src.U(p, s) + (d.r0 - R0);
    g.lda = ld;
    g.B = src.V(p, s) + (d.c0 - C0);
    g.ldb = ld;
    g.opB = 1;
    g.C = d.D;
    g.ldc = (int)d.m;
    g.m = (int)d.m;
    g.n = (int)d.n;
    g.k = std::max(1, src.cap[l]);
    g.kp = src.rk(p, s);
    g.alpha = 1.0;
    g.beta = 0.0;
    gm.push_back(g);
    maxm = std::max<int>(maxm, (int)d.m);
    maxn = std::max<int>(maxn, (int)d.n);
  }
  leaves = src.leaves;  // borrowed from the source HODLR for the export (diagonal blocks)
  ldl = src.ldl;
  e->clear_flags(1);
  e->recompress(rec);
  e->gemm(gm, maxm, maxn);
  const int f = e->read_flags(1)[0];  // synchronises the stream
  if (f & (4 | 8 | 16 | 32)) throw std::runtime_error("hodlr_to_hmatrix: a sub-block recompression failed");
  ranks.assign(lr.size(), 0);
  for (size_t i = 0; i < lr.size(); ++i)
    HQ_CHECK(hipMemcpyAsync(&ranks[i], lr[i].rank, sizeof(int), hipMemcpyDeviceToHost, st));
  HQ_CHECK(hipStreamSynchronize(st));
  e->scratch.reset();
  e->stage.reset();
  bytes = 0;
  max_rank = 0;
  for (size_t i = 0; i < lr.size(); ++i) {
    bytes += (int64_t)(lr[i].m + lr[i].n) * ranks[i] * 8;
    max_rank = std::max(max_rank, ranks[i]);
  }
  for (const Dense& d : dn) bytes += (int64_t)d.m * d.n * 8;
}

}  // namespace hq

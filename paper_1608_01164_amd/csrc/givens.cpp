// Structured Givens QR of [M; I] for a b-banded symmetric M (Sec. 4, Algorithms 1 and 2) and the
// direct HODLR construction of the orthogonal factor (Remark construct_off and Theorems
// ranks_tridiag / ranks_banded).
//
// The rotation sweep is inherently sequential and O(b^2 n); it runs on the host, as in the
// paper.  The Q factors are then assembled block by block:
//  * leaves: the rows [lo, hi) of Q1 and of Q2 are replayed densely from the first step that can
//    touch them (lo - b) to the last step of the leaf (hi - 1);
//  * after step k, the rows 0..k of Q live, outside the finished columns, in the span of the 2b
//    "active" columns {k+1..k+b, n, n+k+1..n+k+b-1} (proof of Theorem ranks_banded), so the
//    upper block of node [lo, hi) = (a, b) is U V^T with U = those active columns restricted to
//    the rows of a at step mid-1, and V the coefficients of the columns of b in that basis,
//    obtained by replaying only the rotations of steps mid..hi-1 on 2b-vectors;
//  * the basis of a parent is the children's bases glued together ([U_a C; U_b]), so nothing of
//    size larger than the block itself is ever formed.
#include "givens.h"


#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "engine.h"

namespace hq {

namespace {

// A row of R kept as a short window of columns [c0, c0 + len), len <= W (entries outside are zero).
struct RowStore {
  int W;
  std::vector<int64_t> c0;
  std::vector<int> len;
  std::vector<double> v;
  double* row(int64_t r) { return v.data() + (size_t)r * W; }
  double get(int64_t r, int64_t col) {
    const int64_t k = col - c0[r];
    return (k >= 0 && k < len[r]) ? v[(size_t)r * W + k] : 0.0;
  }
};

inline void make_rot(double f, double g, double& c, double& s) {
  const double m = std::max(std::fabs(f), std::fabs(g));
  // plain sqrt where neither square can overflow or underflow, hypot's scaling otherwise
  const double r = (m > 1e-150 && m < 1e150) ? std::sqrt(f * f + g * g) : std::hypot(f, g);
  if (r == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    c = f / r;
    s = g / r;
  }
}

}  // namespace

GivensSweep structured_qr(const double* ab, int64_t n, int b, int64_t ldab, double shift, double scale) {
  GivensSweep g;
  // room for every rotation: (2b+1) n - b^2 - b of them for b > 1, 3n - 2 for b = 1
  g.rots.reserve((size_t)n * (2 * b + 2));
  g.step.reserve(n + 1);
  RowStore R;
  R.W = 4 * b + 8;
  const int W = R.W;
  R.c0.assign(2 * n, 0);
  R.len.assign(2 * n, 1);
  R.v.assign((size_t)2 * n * W, 0.0);
  // rows 0..n-1: scale * (A - shift I); window starts at column i - b
  for (int64_t i = 0; i < n; ++i) {
    R.c0[i] = i - b;
    R.len[i] = 2 * b + 1;
    double* r = R.row(i);
    for (int64_t j = std::max<int64_t>(0, i - b); j <= std::min<int64_t>(n - 1, i + b); ++j) {
      const int64_t d = i >= j ? i - j : j - i, col = std::min(i, j);
      double v = ab[d + col * ldab];
      if (i == j) v -= shift;
      r[j - (i - b)] = scale * v;
    }
  }
  // rows n..2n-1: identity rows; row n is the one all beta rotations act on
  for (int64_t i = 0; i < n; ++i) {
    R.c0[n + i] = i;
    R.row(n + i)[0] = 1.0;
  }
  std::vector<double> xp(2 * W), xq(2 * W), tp(2 * W), tq(2 * W);
  auto store = [&](int64_t r, const double* t, int64_t lo, int span) {
    int first = 0, last = span - 1;
    while (first < span && t[first] == 0.0) ++first;
    double* out = R.row(r);
    if (first == span) {
      R.len[r] = 0;
      return;
    }
    while (t[last] == 0.0) --last;
    if (last - first >= W) throw std::runtime_error("structured_qr: row window overflow");
    std::copy(t + first, t + last + 1, out);
    R.c0[r] = lo + first;
    R.len[r] = last - first + 1;
  };
  // rotation in rows (P, Q) chosen so that R(Q, col) becomes zero; both windows are laid side by
  // side over their union [lo, lo + span) and rotated there
  auto rot = [&](int64_t P, int64_t Q, int64_t col) {
    const int64_t cP = R.c0[P], cQ = R.c0[Q];
    const double* rp = R.row(P);
    const double* rq = R.row(Q);
    double c, s;
    make_rot(R.get(P, col), R.get(Q, col), c, s);
    g.rots.push_back({P, Q, c, s});
    const int lP = R.len[P], lQ = R.len[Q];
    const int64_t lo = std::min(lP ? cP : cQ, lQ ? cQ : cP);
    const int span = (int)(std::max(cP + lP, cQ + lQ) - lo);
    std::fill(xp.begin(), xp.begin() + span, 0.0);
    std::fill(xq.begin(), xq.begin() + span, 0.0);
    if (lP) std::copy(rp, rp + lP, xp.begin() + (cP - lo));
    if (lQ) std::copy(rq, rq + lQ, xq.begin() + (cQ - lo));
    for (int k = 0; k < span; ++k) {
      tp[k] = c * xp[k] + s * xq[k];
      tq[k] = -s * xp[k] + c * xq[k];
    }
    if (col >= lo && col < lo + span) tq[col - lo] = 0.0;
    store(P, tp.data(), lo, span);
    store(Q, tq.data(), lo, span);
  };
  for (int64_t i = 0; i < n; ++i) {
    g.step.push_back((int64_t)g.rots.size());
    if (i == 0) {
      rot(0, n, 0);                                                  // beta_1
      for (int64_t j = 1; j <= std::min<int64_t>(n - 1, b); ++j) rot(0, j, 0);  // gamma_{1,j}
      continue;
    }
    rot(n, n + i, i);                                                // alpha_{i,i}
    for (int64_t j = i + 1; j <= std::min<int64_t>(n - 1, b + i - 1); ++j) rot(n + j, n + i, j);  // alpha_{i,j}
    rot(i, n, i);                                                    // beta_i
    if (i < n - 1)
      for (int64_t j = i + 1; j <= std::min<int64_t>(n - 1, b + i); ++j) rot(i, j, i);  // gamma_{i,j}
  }
  g.step.push_back((int64_t)g.rots.size());
  return g;
}

// ---------------------------------------------------------------------------------------------
namespace {

// Active column set after 0-based step k: {k+1..k+b, n, n+k+1..n+k+b-1}; -1 marks a column
// beyond the matrix (its coefficient stays zero).
std::vector<int64_t> active_set(int64_t k, int64_t n, int b) {
  std::vector<int64_t> a;
  for (int j = 1; j <= b; ++j) a.push_back(k + j < n ? k + j : -1);
  a.push_back(n);
  for (int j = 1; j <= b - 1; ++j) a.push_back(k + j < n ? n + k + j : -1);
  return a;
}

// column map for a window [lo0, hi0) of the first n columns, column n, and n + [lo0, hi0)
struct ColMap {
  int64_t n, lo0, w;
  int size() const { return (int)(2 * w + 1); }
  int operator()(int64_t col) const {
    if (col < n) {
      const int64_t k = col - lo0;
      return (k >= 0 && k < w) ? (int)k : -1;
    }
    if (col == n) return (int)w;
    const int64_t k = col - n - lo0;
    return (k >= 0 && k < w) ? (int)(w + 1 + k) : -1;
  }
};

}  // namespace

size_t host_hodlr_doubles(const Tree& t, const std::vector<int>& cap, int ldl) {
  size_t s = (size_t)t.nleaves * ldl * ldl;
  for (int l = 0; l < t.L; ++l) s += 2 * (size_t)(2 << l) * t.ldf[l] * cap[l];
  return s;
}

namespace {
void bind_image(HostHodlr& h, const Tree& t, const std::vector<int>& cap, int ldl, double* mem) {
  h.nleaves = (size_t)t.nleaves * ldl * ldl;
  h.leaves = mem;
  mem += h.nleaves;
  h.U.assign(t.L, nullptr);
  h.V.assign(t.L, nullptr);
  h.fsize.assign(t.L, 0);
  for (int l = 0; l < t.L; ++l) {
    h.fsize[l] = (size_t)(2 << l) * t.ldf[l] * cap[l];
    h.U[l] = mem;
    mem += h.fsize[l];
    h.V[l] = mem;
    mem += h.fsize[l];
  }
  h.rank.assign(std::max(1, 2 * t.ninternal), 0);
}

// Rotate the columns x, y (len rows each) of a column-major block.
inline void apply_rot(const Rot& R, double* x, double* y, int64_t len) {
  for (int64_t r = 0; r < len; ++r) {
    const double u = x[r], w = y[r];
    x[r] = R.c * u + R.s * w;
    y[r] = -R.s * u + R.c * w;
  }
}

}  // namespace

void q_factors_hodlr(const GivensSweep& g, const Tree& t, int b, const std::vector<int>& cap, int ldl,
                     HostHodlr& q1, HostHodlr& q2, double* mem) {
  const int64_t n = t.n;
  const int L = t.L, B2 = 2 * b;
  for (int l = 0; l < L; ++l)
    if (cap[l] < B2) throw std::runtime_error("q_factors_hodlr: capacity below 2b");
  const size_t one = host_hodlr_doubles(t, cap, ldl);
  if (mem) {
    bind_image(q1, t, cap, ldl, mem);
    bind_image(q2, t, cap, ldl, mem + one);
  } else {
    q1.own.assign(one, 0.0);
    q2.own.assign(one, 0.0);
    bind_image(q1, t, cap, ldl, q1.own.data());
    bind_image(q2, t, cap, ldl, q2.own.data());
  }
  if ((int64_t)g.step.size() != n + 1) throw std::runtime_error("q_factors_hodlr: sweep of another size");
  const Rot* const rots = g.rots.data();
  const int64_t* const step = g.step.data();
  // basis of each node's rows (Q1 rows then Q2 rows) x 2b, at the end of the node's last step
  std::vector<std::unique_ptr<double[]>> basis(t.nnodes);
  // lower-left corner of Q1 next to the first leaf of every right subtree: rows lo..lo+b-1, cols lo-b..lo-1
  std::vector<std::vector<double>> corner(t.nleaves);
  // coefficients, after step hi-1, of the active columns at step mid-1 (2b x 2b per internal node)
  std::vector<std::vector<double>> cend(t.ninternal);

  // Leaf replays (dense rows of the leaf) and, for every internal node, the replay of its steps on
  // 2b-vectors: none needs anything but the rotations, so they are independent tasks, run longest
  // first (the top levels' replays, then the lower levels' and the leaves).  Each task also clears
  // the parts of the images it owns, so that every entry is written by one task.
  const int ntask = t.nnodes;

  auto leaf_task = [&](int p) {
    const int li = p - t.ninternal;
    const int64_t lo = t.lo[p], hi = t.hi[p], m = hi - lo;
    ColMap cm{n, lo - b, m + 2 * b};
    const int nc = cm.size();
    const int64_t rows = 2 * m;
    std::vector<double> D((size_t)rows * nc, 0.0);  // column-major rows x nc
    auto at = [&](int64_t r, int c) -> double& { return D[(size_t)c * rows + r]; };
    for (int64_t r = 0; r < m; ++r) {
      at(r, cm(lo + r)) = 1.0;
      at(m + r, cm(n + lo + r)) = 1.0;
    }
    for (int64_t st = std::max<int64_t>(0, lo - b); st < hi; ++st) {
      for (int64_t k = step[st]; k < step[st + 1]; ++k) {
        const Rot& R = rots[k];
        const int ip = cm(R.p), iq = cm(R.q);
        if (ip < 0 || iq < 0) throw std::runtime_error("q_factors_hodlr: leaf window");
        apply_rot(R, &D[(size_t)ip * rows], &D[(size_t)iq * rows], rows);
      }
    }
    double* L1 = q1.leaves + (size_t)li * ldl * ldl;
    double* L2 = q2.leaves + (size_t)li * ldl * ldl;
    std::fill(L1, L1 + (size_t)ldl * ldl, 0.0);
    std::fill(L2, L2 + (size_t)ldl * ldl, 0.0);
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = 0; r < m; ++r) {
        L1[r + c * ldl] = at(r, cm(lo + c));
        L2[r + c * ldl] = at(m + r, cm(lo + c));
      }
    if (lo > 0) {
      corner[li].assign((size_t)b * b, 0.0);
      for (int tr = 0; tr < b; ++tr)
        for (int j = 0; j < b; ++j) corner[li][tr + (size_t)j * b] = at(tr, cm(lo - b + j));
    }
    double* Bs = new double[(size_t)rows * B2];
    basis[p].reset(Bs);
    const std::vector<int64_t> act = active_set(hi - 1, n, b);
    for (int k = 0; k < B2; ++k) {
      const int ic = act[k] < 0 ? -1 : cm(act[k]);
      if (act[k] >= 0 && ic < 0) throw std::runtime_error("q_factors_hodlr: active column outside leaf window");
      for (int64_t r = 0; r < rows; ++r) Bs[(size_t)k * rows + r] = ic < 0 ? 0.0 : at(r, ic);
    }
  };

  auto node_task = [&](int p) {
    const int l = Tree::level(p), i = p - ((1 << l) - 1);
    const int64_t ldf = t.ldf[l];
    const size_t blk = (size_t)ldf * cap[l], off0 = (size_t)(2 * i) * blk;
    for (HostHodlr* h : {&q1, &q2}) {
      std::fill(h->U[l] + off0, h->U[l] + off0 + 2 * blk, 0.0);
      std::fill(h->V[l] + off0, h->V[l] + off0 + 2 * blk, 0.0);
    }
    const int64_t mid = t.mid(p), hi = t.hi[p], mb = hi - mid;
    // coefficient replay over steps mid..hi-1
    ColMap cm{n, mid, (hi - mid) + b + 1};
    const int nc = cm.size();
    std::vector<double> Cf((size_t)B2 * nc, 0.0);  // column c of Q -> 2b coefficients
    const std::vector<int64_t> act0 = active_set(mid - 1, n, b);
    for (int k = 0; k < B2; ++k)
      if (act0[k] >= 0) {
        const int ic = cm(act0[k]);
        if (ic < 0) throw std::runtime_error("q_factors_hodlr: start basis outside window");
        Cf[(size_t)ic * B2 + k] = 1.0;
      }
    for (int64_t st = mid; st < hi; ++st) {
      for (int64_t k = step[st]; k < step[st + 1]; ++k) {
        const Rot& R = rots[k];
        const int ip = cm(R.p), iq = cm(R.q);
        if (ip < 0 || iq < 0) throw std::runtime_error("q_factors_hodlr: node window");
        apply_rot(R, &Cf[(size_t)ip * B2], &Cf[(size_t)iq * B2], B2);
      }
    }
    // V of the upper block: row j - mid = the coefficients of column j (the same for Q1 and Q2)
    for (int k = 0; k < B2; ++k)
      for (int64_t j = 0; j < mb; ++j) {
        const double v = Cf[(size_t)cm(mid + j) * B2 + k];
        q1.V[l][off0 + j + (size_t)k * ldf] = v;
        q2.V[l][off0 + j + (size_t)k * ldf] = v;
      }
    if (p > 0) {  // the parent glues this node's basis from the children's and these coefficients
      const std::vector<int64_t> act1 = active_set(hi - 1, n, b);
      std::vector<double>& Ce = cend[p];
      Ce.assign((size_t)B2 * B2, 0.0);
      for (int k = 0; k < B2; ++k)
        if (act1[k] >= 0) {
          const int ic = cm(act1[k]);
          if (ic < 0) throw std::runtime_error("q_factors_hodlr: end basis outside window");
          for (int r = 0; r < B2; ++r) Ce[(size_t)k * B2 + r] = Cf[(size_t)ic * B2 + r];
        }
    }
  };

  // a failed window check (an exception) must not leave the parallel region: the first is kept and
  // rethrown after it
  std::exception_ptr err;
  std::mutex err_mu;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < ntask; ++p) {
    try {
      if (t.is_leaf(p))
        leaf_task(p);
      else
        node_task(p);
    } catch (...) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (!err) err = std::current_exception();
    }
  }
  if (err) std::rethrow_exception(err);

  // U factors and the bases of internal nodes, bottom-up: per level, one task per (node, column of
  // the 2b-wide basis), copies and 2b-term combinations only
  for (int l = L - 1; l >= 0; --l) {
    const int f0 = (1 << l) - 1, cnt = 1 << l;
    const int64_t ldf = t.ldf[l];
    const size_t blk = (size_t)ldf * cap[l];
    for (int p = std::max(f0, 1); p < f0 + cnt; ++p) basis[p].reset(new double[(size_t)2 * t.size(p) * B2]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int task = 0; task < cnt * B2; ++task) {
      const int p = f0 + task / B2, k = task % B2, i = p - f0;
      const int a = 2 * p + 1, bb = 2 * p + 2;
      const int64_t lo = t.lo[p], mid = t.mid(p), hi = t.hi[p];
      const int64_t ma = mid - lo, mb = hi - mid;
      const double* Ba = basis[a].get();  // (2 ma) x 2b
      const size_t off0 = (size_t)(2 * i) * blk, off1 = off0 + blk;
      // upper blocks: column k of U = column k of a's basis (Q1 part / Q2 part)
      const double* bak = Ba + (size_t)k * 2 * ma;
      std::copy(bak, bak + ma, q1.U[l] + off0 + (size_t)k * ldf);
      std::copy(bak + ma, bak + 2 * ma, q2.U[l] + off0 + (size_t)k * ldf);
      if (k == 0) {
        q1.rank[2 * p] = B2;
        q2.rank[2 * p] = B2;
        // lower block of Q1: the b x b corner rows mid..mid+b-1, cols mid-b..mid-1
        const int lf = (int)(((int64_t)(bb + 1) << (L - l - 1)) - 1) - t.ninternal;  // first leaf under bb
        const std::vector<double>& cr = corner[lf];
        for (int tr = 0; tr < b; ++tr) {
          q1.U[l][off1 + tr + (size_t)tr * ldf] = 1.0;
          for (int j = 0; j < b; ++j) q1.V[l][off1 + (ma - b + j) + (size_t)tr * ldf] = cr[tr + (size_t)j * b];
        }
        q1.rank[2 * p + 1] = b;
        q2.rank[2 * p + 1] = 0;
      }
      // column k of p's basis at the end of step hi-1: [basis(a) Cend(:, k); basis(b)(:, k)] per part
      if (p > 0) {
        const double* ce = cend[p].data() + (size_t)k * B2;
        const double* Bb = basis[bb].get();  // (2 mb) x 2b
        const int64_t rows = 2 * (ma + mb);
        double* bp = basis[p].get() + (size_t)k * rows;
        for (int part = 0; part < 2; ++part) {
          double* o = bp + part * (ma + mb);
          std::fill(o, o + ma, 0.0);
          for (int q = 0; q < B2; ++q) {
            const double c = ce[q];
            const double* src = Ba + (size_t)q * 2 * ma + part * ma;
            for (int64_t r = 0; r < ma; ++r) o[r] += src[r] * c;
          }
          std::copy(Bb + (size_t)k * 2 * mb + part * mb, Bb + (size_t)k * 2 * mb + (part + 1) * mb, o + ma);
        }
      }
    }
    // children bases are no longer needed
    for (int p = f0; p < f0 + cnt; ++p) {
      basis[2 * p + 1].reset();
      basis[2 * p + 2].reset();
    }
  }
}

int64_t q_factors_from_band(const double* ab, int64_t n, int b, int64_t ldab, double shift, double scale,
                            const Tree& t, const std::vector<int>& cap, int ldl, HostHodlr& q1, HostHodlr& q2,
                            double* mem) {
  if (t.n != n) throw std::runtime_error("q_factors_from_band: tree of another size");
  const GivensSweep g = structured_qr(ab, n, b, ldab, shift, scale);
  q_factors_hodlr(g, t, b, cap, ldl, q1, q2, mem);
  return (int64_t)g.rots.size();
}

}  // namespace hq

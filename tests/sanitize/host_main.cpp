// Host parts of the library under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU:
// the cluster tree, the Zolotarev coefficients (Sec. 2.1) and the structured QR sweep of Sec. 4 with
// its HODLR host images, on small random bands (ragged trees, b = 1 and b > 1, n <= leaf).
#include <cmath>
#include <cstdio>
#include <exception>
#include <random>
#include <vector>

#include "../../paper_1608_01164_amd/csrc/engine.h"
#include "../../paper_1608_01164_amd/csrc/givens.h"
#include "../../paper_1608_01164_amd/csrc/zolo.h"

static int failures = 0;
static void check(bool ok, const char* what, double a = 0, double b = 0) {
  if (!ok) {
    std::printf("FAIL %s (%g, %g)\n", what, a, b);
    ++failures;
  }
}

int main() {
  // cluster trees: children split their parent, leaves hold at most `leaf` indices
  const long ns[] = {1, 2, 3, 64, 100, 777, 4096};
  const int leaves[] = {1, 8, 64};
  for (long n : ns)
    for (int leaf : leaves) {
      hq::Tree t;
      t.build(n, leaf);
      check(t.lo[0] == 0 && t.hi[0] == n, "tree root", (double)n, leaf);
      for (int p = 0; p < t.ninternal; ++p)
        check(t.lo[2 * p + 1] == t.lo[p] && t.hi[2 * p + 1] == t.lo[2 * p + 2] && t.hi[2 * p + 2] == t.hi[p],
              "tree split", (double)n, p);
      for (int p = t.ninternal; p < t.nnodes; ++p) check(t.size(p) <= leaf, "leaf size", (double)n, leaf);
      for (int l = 0; l < t.L; ++l)
        for (int p = (1 << l) - 1; p < (2 << l) - 1; ++p)
          check(t.ldf[l] >= t.size(2 * p + 1) && t.ldf[l] >= t.size(2 * p + 2), "ldf", (double)n, l);
    }
  // Zolotarev steps: c[1..2r] positive and increasing, a[1..r] positive (1-based arrays), and the
  // next lower bound in (l, 1]
  const double ls[] = {1e-14, 1e-6, 1e-2, 0.3, 0.9};
  for (double l : ls)
    for (int r = 1; r <= 8; ++r) {
      const hq::ZoloStep z = hq::zolo_step(l, r);
      check((int)z.c.size() == 2 * r + 1 && (int)z.a.size() == r + 1, "zolo sizes", l, r);
      for (int i = 1; i <= 2 * r; ++i) check(std::isfinite(z.c[i]) && z.c[i] > 0, "zolo c", l, i);
      for (int i = 2; i <= 2 * r; ++i) check(z.c[i] > z.c[i - 1], "zolo c order", l, i);
      for (int j = 1; j <= r; ++j) check(std::isfinite(z.a[j]) && z.a[j] > 0, "zolo a", l, j);
      check(std::isfinite(z.mhat) && z.mhat > 0, "zolo mhat", l, r);
      check(z.lnext >= l && z.lnext <= 1.0, "zolo lnext", l, z.lnext);
    }
  check(!hq::zolo_schedule(1e-10, 1e-15, 0, 6).empty(), "zolo schedule");
  // structured QR sweep and the HODLR images of Q1, Q2
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  struct Case { long n; int b, leaf; };
  const Case cases[] = {{64, 1, 16}, {300, 3, 32}, {777, 8, 64}, {50, 8, 64}, {129, 2, 8}};
  for (const Case& c : cases) {
    const long ldab = c.b + 1;
    std::vector<double> ab((size_t)ldab * c.n);
    for (double& x : ab) x = nd(rng);
    hq::Tree t;
    t.build(c.n, c.leaf);
    const std::vector<int> cap(t.L, 2 * c.b);
    hq::HostHodlr q1, q2;
    try {
      const long nr = (long)hq::q_factors_from_band(ab.data(), c.n, c.b, ldab, 0.1, 0.5, t, cap, (int)t.maxleaf, q1, q2);
      check(nr > 0, "rotations", (double)c.n, c.b);
      for (double x : q1.own) check(std::isfinite(x), "Q1 finite", (double)c.n, c.b);
      for (double x : q2.own) check(std::isfinite(x), "Q2 finite", (double)c.n, c.b);
      for (int r : q1.rank) check(r >= 0 && r <= 2 * c.b, "Q1 rank", (double)c.n, r);
    } catch (const std::exception& e) {
      std::printf("FAIL exception %s\n", e.what());
      ++failures;
    }
  }
  std::printf(failures ? "failed %d\n" : "ok\n", failures);
  return failures ? 1 : 0;
}

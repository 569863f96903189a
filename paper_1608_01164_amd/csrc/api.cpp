// C ABI of the library and the hQDWH driver (Algorithm 3 of the paper).
#include "../../include/hq.h"

#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "engine.h"
#include "givens.h"
#include "handle.h"
#include "hmatrix.h"
#include "predictor.h"
#include "zolo.h"


namespace {

thread_local std::string g_err;

hq_status fail(hq_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace

void hq::set_last_error(const std::string& m) { g_err = m; }

namespace {

template <class F>
hq_status guard(F&& f) {
  try {
    return f();
  } catch (const hq::HipError& e) {
    return fail(HQ_ERR_DEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HQ_ERR_ALLOC, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HQ_ERR_DEVICE, e.what());
  }
}

using clk = std::chrono::steady_clock;

// Mixed precision: truncation tolerance of the FP64 iterations that follow FP32 ones (at least opts.tol).
constexpr double kTolAfterFp32 = 1e-8;
double secs(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }

// ---- host setup: alpha, l0, weights ---------------------------------------------------------

// Number of eigenvalues below sigma: negative pivots of the symmetric elimination of A - sigma I,
// carried as a sliding (b+1) x (b+1) trailing block (Sylvester's law of inertia).
int64_t inertia_below(const double* ab, int64_t n, int b, int64_t ld, double sigma, double pivmin,
                      std::vector<double>& S) {
  int64_t neg = 0;
  if (b > 63) throw std::runtime_error("inertia count supports b <= 63");
  if (b == 1) {
    double q = 1.0;
    for (int64_t i = 0; i < n; ++i) {
      const double e = i > 0 ? ab[1 + (i - 1) * ld] : 0.0;
      q = (ab[i * ld] - sigma) - (i > 0 ? e * e / q : 0.0);
      if (std::fabs(q) < pivmin) q = -pivmin;
      neg += q < 0.0;
    }
    return neg;
  }
  const int w = b + 1;
  S.assign((size_t)w * w, 0.0);  // S(r, c), r, c in window rows j..j+b (symmetric, lower used)
  auto A = [&](int64_t i, int64_t j) -> double {  // i >= j, i - j <= b
    return ab[(i - j) + j * ld] - (i == j ? sigma : 0.0);
  };
  for (int r = 0; r < w && r < n; ++r)
    for (int c = 0; c <= r; ++c) S[r + (size_t)c * w] = A(r, c);
  for (int64_t j = 0; j < n; ++j) {
    double d = S[0];
    if (std::fabs(d) < pivmin) d = -pivmin;
    neg += d < 0.0;
    const int act = (int)std::min<int64_t>(b, n - 1 - j);  // live rows below the pivot
    // Schur update of the trailing block, shifted up-left by one
    double col[64];
    for (int r = 0; r < act; ++r) col[r] = S[r + 1];
    for (int c = 0; c < act; ++c) {
      const double lc = col[c] / d;
      for (int r = c; r < act; ++r) S[r + (size_t)c * w] = S[(r + 1) + (size_t)(c + 1) * w] - col[r] * lc;
    }
    // new last row/col from A
    if (j + 1 + b < n) {
      const int64_t ni = j + 1 + b;
      for (int c = 0; c <= b; ++c) S[b + (size_t)c * w] = (ni - (j + 1 + c) <= b) ? A(ni, j + 1 + c) : 0.0;
    }
  }
  return neg;
}

double pivmin_of(const double* ab, int64_t n, int b, int64_t ld) {
  double m = 1.0;
  for (int64_t j = 0; j < n; ++j)
    for (int i = 1; i <= b && j + i < n; ++i) m = std::max(m, ab[i + j * ld] * ab[i + j * ld]);
  return 2.2250738585072014e-308 * m;
}

double norm_inf_shifted(const double* ab, int64_t n, int b, int64_t ld, double mu) {
  std::vector<double> rs(n, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    rs[j] += std::fabs(ab[j * ld] - mu);
    for (int i = 1; i <= b && j + i < n; ++i) {
      const double v = std::fabs(ab[i + j * ld]);
      rs[j] += v;
      rs[j + i] += v;
    }
  }
  double m = 0.0;
  for (double v : rs) m = std::max(m, v);
  return m;
}

// Largest delta = alpha 2^-k with no eigenvalue in [mu - delta, mu + delta): a certified lower bound
// of dist(mu, spectrum) within a factor of two.  Returns 0 if none down to 1e-15 alpha.
double certified_distance(const double* ab, int64_t n, int b, int64_t ld, double mu, double alpha) {
  const double pm = pivmin_of(ab, n, b, ld);
  std::vector<double> S;
  const int64_t nu = inertia_below(ab, n, b, ld, mu, pm, S);
  const int K = 52;
  std::vector<int> ok(K + 1, 0);
  int found = -1;
  for (int k0 = 1; k0 <= K && found < 0; k0 += 8) {
    const int k1 = std::min(K, k0 + 7);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = k0; k <= k1; ++k) {
      std::vector<double> SS;
      const double d = std::ldexp(alpha, -k);
      ok[k] = inertia_below(ab, n, b, ld, mu - d, pm, SS) == nu && inertia_below(ab, n, b, ld, mu + d, pm, SS) == nu;
    }
    for (int k = k0; k <= k1; ++k)
      if (ok[k]) {
        found = k;
        break;
      }
  }
  if (found < 0) return 0.0;
  return std::ldexp(alpha, -found);
}

double h_of(double l) {
  const double l2 = l * l;
  const double g = std::cbrt(4.0 * (1.0 - l2) / (l2 * l2));
  const double sg = std::sqrt(1.0 + g);
  return sg + 0.5 * std::sqrt(8.0 - 4.0 * g + 8.0 * (2.0 - l2) / (l2 * sg));
}

struct Weights {
  std::vector<double> a, b, c;
  double lK;
};
Weights schedule(double l0, double delta, int max_iter) {
  Weights w;
  double l = l0;
  while (std::fabs(1.0 - l) > delta && (int)w.a.size() < max_iter) {
    const double a = h_of(l), b = (a - 1.0) * (a - 1.0) / 4.0, c = a + b - 1.0;
    w.a.push_back(a);
    w.b.push_back(b);
    w.c.push_back(c);
    l = l * (a + b * l * l) / (1.0 + c * l * l);
    if (l > 1.0) l = 1.0;
  }
  w.lK = l;
  return w;
}

// ---- helpers --------------------------------------------------------------------------------

std::vector<int> caps_from(const hq::Tree& t, int v, int maxr) {
  std::vector<int> c(t.L);
  for (int l = 0; l < t.L; ++l) c[l] = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)v, (int64_t)maxr, t.ldf[l]}));
  return c;
}

std::vector<int> caps_grow(const hq::Tree& t, const std::vector<int>& ranks, int maxr, int mult, int add) {
  std::vector<int> c(t.L, 1);
  for (int p = 0; p < t.ninternal; ++p) {
    const int l = hq::Tree::level(p);
    c[l] = std::max(c[l], std::max(ranks[2 * p], ranks[2 * p + 1]));
  }
  for (int l = 0; l < t.L; ++l)
    c[l] = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)c[l] * mult + add, (int64_t)maxr, t.ldf[l]}));
  return c;
}

int max_of(const std::vector<int>& v) {
  int m = 0;
  for (int x : v) m = std::max(m, x);
  return m;
}

void upload_host(hq::Engine& e, const hq::HostHodlr& h, hq::HMat& H, bool sync = true) {
  const hq::Tree& t = *H.t;
  HQ_CHECK(hipMemcpyAsync(H.leaves, h.leaves, sizeof(double) * h.nleaves, hipMemcpyHostToDevice, e.st));
  for (int l = 0; l < t.L; ++l) {
    HQ_CHECK(hipMemcpyAsync(H.Ubase[l], h.U[l], sizeof(double) * h.fsize[l], hipMemcpyHostToDevice, e.st));
    HQ_CHECK(hipMemcpyAsync(H.Vbase[l], h.V[l], sizeof(double) * h.fsize[l], hipMemcpyHostToDevice, e.st));
  }
  if (t.ninternal > 0)
    HQ_CHECK(hipMemcpyAsync(H.rank, h.rank.data(), sizeof(int) * 2 * t.ninternal, hipMemcpyHostToDevice, e.st));
  if (sync) HQ_CHECK(hipStreamSynchronize(e.st));  // host buffers go out of scope
}

// X0 = (A - shift I) * inv_scale directly from the device band.
void build_x0(hq::Engine& e, const double* band, int64_t n, int b, int64_t ldab, double shift, double inv_scale,
              hq::HMat& X) {
  const hq::Tree& t = *X.t;
  hq::BandDesc bd{band, n, ldab, b, shift, inv_scale};
  std::vector<int64_t> lo(t.nleaves);
  std::vector<int> ms(t.nleaves);
  for (int i = 0; i < t.nleaves; ++i) {
    lo[i] = t.lo[t.ninternal + i];
    ms[i] = (int)t.size(t.ninternal + i);
  }
  hq::launch_band_leaves(bd, X.leaves, X.ldl, e.stage.upload(lo, e.st), e.stage.upload(ms, e.st), t.nleaves, e.st);
  std::vector<hq::BandBlockTask> bt;
  int maxrows = 1;
  for (int p = 0; p < t.ninternal; ++p) {
    hq::BandBlockTask k{};
    k.Ul = X.U(p, 1);
    k.Vl = X.V(p, 1);
    k.Uu = X.U(p, 0);
    k.Vu = X.V(p, 0);
    k.rank_l = X.rk(p, 1);
    k.rank_u = X.rk(p, 0);
    k.mid = t.mid(p);
    k.rows_a = (int)t.size(2 * p + 1);
    k.rows_b = (int)t.size(2 * p + 2);
    k.ldf = X.ld(p);
    maxrows = std::max({maxrows, k.rows_a, k.rows_b});
    bt.push_back(k);
  }
  hq::launch_band_blocks(bd, e.stage.upload(bt, e.st), (int)bt.size(), maxrows, e.st);
}

// Copy H (engine E) into a fresh handle whose capacities equal the realised ranks.
hq_hodlr_t compact_copy(hq::Engine& E, const hq::HMat& H, hipStream_t st, int leaf) {
  std::unique_ptr<hq_hodlr_s> h(new hq_hodlr_s());
  h->t.build(H.t->n, leaf);
  const hq::Tree& t = h->t;
  const std::vector<int> r = E.read_ranks(H);
  std::vector<int> cap(t.L, 1);
  for (int p = 0; p < t.ninternal; ++p) {
    const int l = hq::Tree::level(p);
    cap[l] = std::max(cap[l], std::max(r[2 * p], r[2 * p + 1]));
  }
  h->e.reset(new hq::Engine(st));
  h->e->tol = E.tol;
  h->e->persist.chunk_bytes = std::max<size_t>(size_t(1) << 20, H.bytes() + (size_t(4) << 20));
  h->H = h->e->alloc_hmat(&h->t, cap, H.lower_only);
  HQ_CHECK(hipMemcpy2DAsync(h->H.leaves, sizeof(double) * h->H.ldl, H.leaves, sizeof(double) * H.ldl,
                            sizeof(double) * H.ldl, (size_t)t.nleaves * H.ldl, hipMemcpyDeviceToDevice, st));
  std::vector<hq::StackTask> cp;
  int maxrows = 1;
  for (int p = 0; p < t.ninternal; ++p)
    for (int s = 0; s < 2; ++s)
      for (int uv = 0; uv < 2; ++uv) {
        const int rows = (int)((uv == 0) == (s == 0) ? t.size(2 * p + 1) : t.size(2 * p + 2));
        hq::StackTask k{};
        k.dst = uv == 0 ? h->H.U(p, s) : h->H.V(p, s);
        k.ld = h->H.ld(p);
        k.rows = rows;
        k.wcap = h->H.capof(p);
        k.wout = uv == 0 ? h->H.rk(p, s) : nullptr;
        k.nsrc = 1;
        k.src[0] = {uv == 0 ? H.U(p, s) : H.V(p, s), H.rk(p, s), H.ld(p), H.capof(p), 1.0};
        cp.push_back(k);
        maxrows = std::max(maxrows, rows);
      }
  if (!cp.empty()) h->e->stack(cp, maxrows);
  HQ_CHECK(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  h->d_w = h->e->persist.get<int>(1);
  HQ_CHECK(hipStreamSynchronize(st));
  h->e->stage.reset();
  reserve_apply_staging(*h);
  return h.release();
}

hq_status check_opts(const hq_opts* o, hq_opts& out) {
  hq_default_opts(&out);
  if (o) out = *o;
  if (out.leaf < 2) return fail(HQ_ERR_ARG, "opts.leaf must be >= 2");
  if (!(out.tol > 0.0)) return fail(HQ_ERR_ARG, "opts.tol must be > 0");
  if (!(out.delta > 0.0)) return fail(HQ_ERR_ARG, "opts.delta must be > 0");
  if (out.max_rank < 1) return fail(HQ_ERR_ARG, "opts.max_rank must be >= 1");
  if (out.max_iter < 1 || out.max_iter > 16) return fail(HQ_ERR_ARG, "opts.max_iter must be in [1, 16]");
  if (out.precision != HQ_FP64 && out.precision != HQ_MIXED) return fail(HQ_ERR_ARG, "opts.precision must be FP64 or MIXED");
  if (out.method != HQ_METHOD_QDWH && out.method != HQ_METHOD_ZOLO) return fail(HQ_ERR_ARG, "opts.method must be QDWH or ZOLO");
  if (out.zolo_r < 0 || out.zolo_r > 8) return fail(HQ_ERR_ARG, "opts.zolo_r must be in [0, 8]");
  if (out.graph)
    return fail(HQ_ERR_UNSUPPORTED,
                "opts.graph: launching an iteration as a captured HIP graph is disabled (the capture "
                "path ended its first test run in a host segmentation fault whose cause is not found)");
  return HQ_OK;
}

hq_status check_band(const double* band, int64_t n, int32_t b, int64_t ldab) {
  if (!band) return fail(HQ_ERR_ARG, "band is NULL");
  if (n < 1) return fail(HQ_ERR_ARG, "n must be >= 1");
  if (b < 1) return fail(HQ_ERR_ARG, "b must be >= 1");
  if (ldab < b + 1) return fail(HQ_ERR_ARG, "ldab must be >= b+1");
  return HQ_OK;
}

// ---- the hQDWH driver -----------------------------------------------------------------------
// One member of a (possibly singleton) batch of independent problems.  All members share the
// engine, the stream and every kernel launch; each keeps its own tree, weights and capacities.
struct Member {
  const double* band = nullptr;
  int64_t n = 0, ldab = 0;
  int b = 0, beff = 0;
  double mu = 0.0;
  hq_status status = HQ_OK;
  std::string err;
  hq::Tree t;
  std::vector<double> ab;  // host copy of the band
  Weights w;
  int K = 0;
  hq_info inf;
  hq::HMat X, Xn, Z, Linv, Lf, Y, Q1, Q2, P;
  std::vector<int> capX, capZ, capL, capY;  // capacities of X_{k+1}, Z, L and L^{-1}, Y
  std::vector<std::array<std::vector<int>, 4>> pcap;  // predicted capacities per iteration
  bool pred_miss = false;  // an iteration overflowed its predicted capacities
  hq_hodlr_t out = nullptr;
};

std::vector<int> level_max(const hq::Tree& t, const std::vector<int>& r) {
  std::vector<int> m(t.L, 0);
  for (int p = 0; p < t.ninternal; ++p) {
    const int l = hq::Tree::level(p);
    m[l] = std::max(m[l], std::max(r[2 * p], r[2 * p + 1]));
  }
  return m;
}

int64_t capacity_columns(const hq::Tree& t, const std::vector<int>& cap) {
  int64_t c = 0;
  for (int l = 0; l < t.L; ++l) c += (int64_t)(2 << l) * cap[l];
  return c;
}

// Capacities of every iteration from the predictor: rows (k, member, level) on a full grid, one
// forward launch per iteration (the previous-rank feature of iteration k is read on the device from
// iteration k-1's output), and a single readback.
void predict_capacities(std::vector<Member>& ms, const hq_opts& o, hipStream_t st, hq::Engine& E) {
  const int nm = (int)ms.size();
  int Kmax = 0, Lmax = 0;
  for (Member& m : ms)
    if (m.status == HQ_OK) {
      Kmax = std::max(Kmax, m.K);
      Lmax = std::max(Lmax, m.t.L);
    }
  for (Member& m : ms)
    if (m.status == HQ_OK) m.pcap.assign(m.K, {});  // members without levels keep empty capacities
  if (Kmax == 0 || Lmax == 0) return;
  const int64_t R = (int64_t)nm * Lmax;
  constexpr int F = hq::kMlpFeatures, O = hq::kMlpOutputs;
  std::vector<float> X((size_t)Kmax * R * F, 0.0f);
  for (int k = 0; k < Kmax; ++k)
    for (int i = 0; i < nm; ++i) {
      const Member& m = ms[i];
      if (m.status != HQ_OK || k >= m.K) continue;
      for (int l = 0; l < m.t.L; ++l)
        hq::predictor_features(&X[((size_t)k * R + (size_t)i * Lmax + l) * F], m.n, m.beff, l, m.t.ldf[l], k,
                               m.w.a[k], m.w.c[k], m.beff, m.inf.l0, o.tol);
    }
  float* dX = E.scratch.get<float>(X.size());
  float* dY = E.scratch.get<float>((size_t)Kmax * R * O);
  HQ_CHECK(hipMemcpyAsync(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, st));
  for (int k = 0; k < Kmax; ++k)
    hq::launch_mlp_forward(o.predictor->d_params, dX + (size_t)k * R * F, k == 0 ? nullptr : dY + (size_t)(k - 1) * R * O,
                           dY + (size_t)k * R * O, R, st);
  std::vector<float> Y((size_t)Kmax * R * O);
  HQ_CHECK(hipMemcpyAsync(Y.data(), dY, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, st));
  HQ_CHECK(hipStreamSynchronize(st));
  for (int i = 0; i < nm; ++i) {
    Member& m = ms[i];
    if (m.status != HQ_OK) continue;
    for (int k = 1; k < m.K; ++k)
      for (int q = 0; q < O; ++q) {
        std::vector<int>& c = m.pcap[k][q];
        c.resize(m.t.L);
        for (int l = 0; l < m.t.L; ++l)
          c[l] = hq::predictor_capacity(Y[((size_t)k * R + (size_t)i * Lmax + l) * O + q], o.predictor->margin[q],
                                        std::min<int64_t>(o.max_rank, m.t.ldf[l]));
      }
  }
}

void set_fail(Member& m, hq_status s, const char* msg) {
  m.status = s;
  m.err = msg;
}

std::vector<std::vector<int>> read_ranks_many(hq::Engine& E, const std::vector<const hq::HMat*>& hs) {
  std::vector<std::vector<int>> r(hs.size());
  for (size_t i = 0; i < hs.size(); ++i) {
    r[i].assign(std::max(1, 2 * hs[i]->t->ninternal), 0);
    HQ_CHECK(hipMemcpyAsync(r[i].data(), hs[i]->rank, sizeof(int) * r[i].size(), hipMemcpyDeviceToHost, E.st));
  }
  HQ_CHECK(hipStreamSynchronize(E.st));
  return r;
}

// Algorithm 3 for every member: setup (line 1), X0, the structured QR step (k = 0), Cholesky
// steps (k >= 1) and the symmetrised result.  Members leave the batch when their own weight
// schedule ends; a capacity overflow repeats the step for the members it hit.
void run_batch(std::vector<Member>& ms, const hq_opts& o, hipStream_t st, bool projector) {
  const auto t0 = clk::now();
  const int nm = (int)ms.size();
  if (nm > hq::Engine::kFlagSlots) throw std::runtime_error("batch larger than the engine's status slots");
  // host copies of the bands
  for (Member& m : ms) {
    m.ab.resize((size_t)m.n * m.ldab);
    HQ_CHECK(hipMemcpyAsync(m.ab.data(), m.band, sizeof(double) * m.ab.size(), hipMemcpyDeviceToHost, st));
  }
  HQ_CHECK(hipStreamSynchronize(st));
  // Alg. 3 line 1: alpha >= ||A - mu I||_2, l0 <= sigma_min(X0), the weight schedule
#pragma omp parallel for schedule(dynamic, 1) if (nm > 1)
  for (int i = 0; i < nm; ++i) {
    Member& m = ms[i];
    const auto ts = clk::now();
    std::memset(&m.inf, 0, sizeof(m.inf));
    m.t.build(m.n, o.leaf);
    if (m.t.L > 0 && (int64_t)m.b > m.n / (int64_t(1) << m.t.L)) {
      set_fail(m, HQ_ERR_UNSUPPORTED, "bandwidth exceeds the smallest diagonal block; raise opts.leaf");
      continue;
    }
    m.beff = (int)std::min<int64_t>(m.b, std::max<int64_t>(1, m.n - 1));
    const double alpha = norm_inf_shifted(m.ab.data(), m.n, m.beff, m.ldab, m.mu);
    if (!(alpha > 0.0)) {
      set_fail(m, HQ_ERR_SINGULAR_SHIFT, "A - mu I is zero");
      continue;
    }
    const double dist = certified_distance(m.ab.data(), m.n, m.beff, m.ldab, m.mu, alpha);
    if (!(dist > 0.0)) {
      set_fail(m, HQ_ERR_SINGULAR_SHIFT, "mu is numerically an eigenvalue of A");
      continue;
    }
    m.w = schedule(dist / alpha, o.delta, o.max_iter);
    if (std::fabs(1.0 - m.w.lK) > o.delta) {
      set_fail(m, HQ_ERR_NO_CONVERGENCE, "weight recurrence did not reach 1 - delta");
      continue;
    }
    m.K = (int)m.w.a.size();
    m.inf.alpha = alpha;
    m.inf.l0 = dist / alpha;
    m.inf.iters = m.K;
    for (int k = 0; k < m.K && k < 16; ++k) {
      m.inf.a[k] = m.w.a[k];
      m.inf.b[k] = m.w.b[k];
      m.inf.c[k] = m.w.c[k];
    }
    m.inf.setup_seconds = secs(ts);
  }
  int Kmax = 0;
  for (Member& m : ms)
    if (m.status == HQ_OK) {
      Kmax = std::max(Kmax, m.K);
      m.inf.levels = m.t.L;
    }

  std::unique_ptr<hq::PinnedHost> qimg;  // host images of Q1, Q2 (read by copies on the stream)
  // Q1, Q2 of the structured QR on the host; their rank arrays are pageable and read by copies on
  // the stream, so they outlive the stream's drain below (declared before it, destroyed after it)
  std::vector<hq::HostHodlr> h1, h2;
  hq::Engine E(st);
  E.tol = o.tol;
  hq::DevArena xa[2], it, qa, pa;
  struct Drain {  // destroyed first: on an early exit the stream drains before any buffer is freed
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{st};
  size_t peak = 0;
  auto note_peak = [&] {
    peak = std::max(peak, E.persist.high_water() + E.scratch.high_water() + E.side_high_water() +
                              xa[0].high_water() + xa[1].high_water() + it.high_water() + qa.high_water() +
                              pa.high_water());
  };
  if (o.predictor) {
    predict_capacities(ms, o, st, E);
    E.scratch.reset();
  }
  int cur = 0;
  for (Member& m : ms) {
    if (m.status != HQ_OK) continue;
    m.X = E.alloc_hmat_in(xa[cur], &m.t, caps_from(m.t, m.beff, o.max_rank), false);
    build_x0(E, m.band, m.n, m.beff, m.ldab, m.mu, 1.0 / m.inf.alpha, m.X);
  }
  std::vector<Member*> done;
  for (int k = 0; k < Kmax; ++k) {
    std::vector<int> act;
    for (int i = 0; i < nm; ++i)
      if (ms[i].status == HQ_OK && k < ms[i].K) act.push_back(i);
    if (act.empty()) break;
    const auto tk = clk::now();
    if (k == 0) {
      for (int i : act) ms[i].capX = caps_from(ms[i].t, 3 * ms[i].beff + 8, o.max_rank);
      // Alg. 3 lines 7-8: structured QR of [sqrt(c0) X0; I] (Algorithms 1/2) and Q1, Q2 in HODLR,
      // built in place in pinned memory (kept until the call ends) and copied from there
      const auto tg = clk::now();
      h1.assign(act.size(), hq::HostHodlr());
      h2.assign(act.size(), hq::HostHodlr());
      std::vector<size_t> qoff(act.size() + 1, 0);
      for (size_t j = 0; j < act.size(); ++j) {
        const Member& m = ms[act[j]];
        qoff[j + 1] = qoff[j] + 2 * hq::host_hodlr_doubles(m.t, std::vector<int>(m.t.L, 2 * m.beff), (int)m.t.maxleaf);
      }
      qimg.reset(new hq::PinnedHost(sizeof(double) * qoff.back()));
#pragma omp parallel for schedule(dynamic, 1) if (act.size() > 1)
      for (int j = 0; j < (int)act.size(); ++j) {
        Member& m = ms[act[j]];
        const auto tj = clk::now();
        const std::vector<int> capQ(m.t.L, 2 * m.beff);
        hq::q_factors_from_band(m.ab.data(), m.n, m.beff, m.ldab, m.mu, std::sqrt(m.w.c[0]) / m.inf.alpha, m.t,
                                capQ, (int)m.t.maxleaf, h1[j], h2[j], qimg->as<double>() + qoff[j]);
        m.inf.givens_seconds = secs(tj);
      }
      // The setup launches have long finished by now; the drained stream lets the iteration below
      // reuse the descriptor stage, while the copies of the images overlap the next host work.
      HQ_CHECK(hipStreamSynchronize(st));
      for (size_t j = 0; j < act.size(); ++j) {
        Member& m = ms[act[j]];
        const std::vector<int> capQ(m.t.L, 2 * m.beff);
        m.Q1 = E.alloc_hmat_in(qa, &m.t, capQ, false);
        m.Q2 = E.alloc_hmat_in(qa, &m.t, capQ, false);
        upload_host(E, h1[j], m.Q1, false);
        upload_host(E, h2[j], m.Q2, false);
      }
      if (act.size() > 1)
        for (int i : act) ms[i].inf.givens_seconds = secs(tg);
    } else if (o.predictor) {
      // A member whose predicted capacities overflowed once gets, from then on, at least the
      // capacities the previous iterate's ranks call for (one rank readback for those members), so
      // that a predictor that under-estimates a problem costs at most one repeated iteration.  The
      // network is trained on FP64 solves: in the mixed mode the FP32 iterations and those after
      // them get the same treatment from the first FP32 iteration on.
      for (int i : act) {
        Member& m = ms[i];
        if (o.precision == HQ_MIXED && k + 1 < m.K && m.w.c[k] <= o.c_fp32_max) m.pred_miss = true;
      }
      std::vector<const hq::HMat*> xs;
      std::vector<int> miss;
      for (int i : act)
        if (ms[i].pred_miss) {
          xs.push_back(&ms[i].X);
          miss.push_back(i);
        }
      const std::vector<std::vector<int>> rk = xs.empty() ? std::vector<std::vector<int>>() : read_ranks_many(E, xs);
      for (int i : act) {
        Member& m = ms[i];
        m.capX = m.pcap[k][0];
        m.capZ = m.pcap[k][1];
        m.capL = m.pcap[k][2];
        m.capY = m.pcap[k][3];
      }
      for (size_t j = 0; j < miss.size(); ++j) {
        Member& m = ms[miss[j]];
        const std::vector<int> g = caps_grow(m.t, rk[j], o.max_rank, 2, 16);
        for (std::vector<int>* cv : {&m.capX, &m.capZ, &m.capL, &m.capY})
          for (int l = 0; l < m.t.L && l < (int)cv->size(); ++l) (*cv)[l] = std::max((*cv)[l], g[l]);
      }
    } else {
      std::vector<const hq::HMat*> xs;
      for (int i : act) xs.push_back(&ms[i].X);
      const std::vector<std::vector<int>> rk = read_ranks_many(E, xs);
      for (size_t j = 0; j < act.size(); ++j) {
        Member& m = ms[act[j]];
        m.capX = m.capZ = m.capL = m.capY = caps_grow(m.t, rk[j], o.max_rank, 2, 16);
      }
    }
    std::vector<int> pend = act;
    xa[cur ^ 1].reset();
    for (int attempt = 0; !pend.empty(); ++attempt) {
      E.stage.reset();
      E.scratch.reset();
      it.reset();
      for (int i : pend) {
        ms[i].Xn = E.alloc_hmat_in(xa[cur ^ 1], &ms[i].t, ms[i].capX, false);
        ms[i].inf.capacity_columns += capacity_columns(ms[i].t, ms[i].capX);
      }
      // a Cholesky iteration as one graph: everything from here to the status readback
      const bool capture = o.graph && k > 0;
      hq::Engine::Graph graph;
      if (capture) E.capture_begin();
      E.clear_flags(nm);
      if (k == 0) {
        // Alg. 3 line 9: X1 = b0/c0 X0 + (a0 - b0/c0)/sqrt(c0) Q1 Q2^T
        std::vector<hq::Engine::ProdTask> pv;
        for (int i : pend) {
          Member& m = ms[i];
          const double a = m.w.a[0], bb = m.w.b[0], c = m.w.c[0];
          hq::Engine::ProdTask q;
          q.A = E.view(m.Q1);
          q.B = E.view(m.Q2, true);
          q.D = E.view(m.X);
          q.alpha = (a - bb / c) / std::sqrt(c);
          q.delta = bb / c;
          q.C = &m.Xn;
          q.fidx = i;
          pv.push_back(q);
        }
        E.product(pv);
      } else {
        // Alg. 3 lines 11-14: W = chol(I + c X^T X); Y W = X; V W^T = Y; X+ = b/c X + (a - b/c) V.
        // Members whose iteration runs in FP32 (mixed mode) go in their own launches, and so do the
        // FP64 iterations that follow FP32 ones: those truncate at max(tol, kTolAfterFp32), since the
        // iterate already carries the FP32 iterations' perturbation (orders of magnitude above it)
        // and a finer truncation would only keep that noise as rank.
        std::vector<int> grp[3];
        for (int i : pend) {
          const Member& m = ms[i];
          const bool f32 = o.precision == HQ_MIXED && k + 1 < m.K && m.w.c[k] <= o.c_fp32_max;
          bool after = false;
          for (int j = 0; j < k && j < 16; ++j) after |= m.inf.fp32_iter[j] != 0;
          grp[f32 ? 1 : (after ? 2 : 0)].push_back(i);
        }
        for (int g = 0; g < 3; ++g) {
        if (grp[g].empty()) continue;
        E.fp32 = g == 1;
        E.tol = g == 2 ? std::max(o.tol, kTolAfterFp32) : o.tol;
        if (g == 1 && k < 16)
          for (int i : grp[g]) ms[i].inf.fp32_iter[k] = 1;
        std::vector<hq::Engine::ProdTask> pz, py, px;
        std::vector<hq::Engine::CholTask> pc;
        for (int i : grp[g]) {
          Member& m = ms[i];
          m.Z = E.alloc_hmat_in(it, &m.t, m.capZ, true);
          m.Linv = E.alloc_hmat_in(it, &m.t, m.capL, false);
          const int capS = 2 * max_of(m.capL) + 16;
          const std::vector<int> capW = E.chol_work_caps(m.t, m.capZ, capS);
          m.Lf = E.alloc_hmat_in(it, &m.t, capW, false);
          m.Y = E.alloc_hmat_in(it, &m.t, m.capY, false);
          m.inf.capacity_columns += capacity_columns(m.t, m.capZ) / 2 + capacity_columns(m.t, m.capL) +
                                    capacity_columns(m.t, capW) + capacity_columns(m.t, m.capY);
          const double a = m.w.a[k], bb = m.w.b[k], c = m.w.c[k];
          hq::Engine::ProdTask q;
          q.A = E.view(m.X, true);
          q.B = E.view(m.X);
          q.d_identity = true;
          q.alpha = c;
          q.delta = 1.0;
          q.C = &m.Z;
          q.fidx = i;
          pz.push_back(q);
          pc.push_back(hq::Engine::CholTask{&m.Z, &m.Linv, &m.Lf, capS, i});
          q = hq::Engine::ProdTask{};
          q.A = E.view(m.X);
          q.B = E.view(m.Linv, true);  // Y = X L^{-T} = X W^{-1}
          q.C = &m.Y;
          q.fidx = i;
          py.push_back(q);
          q = hq::Engine::ProdTask{};
          q.A = E.view(m.Y);
          q.B = E.view(m.Linv);  // V = Y L^{-1} = Y W^{-T}
          q.D = E.view(m.X);
          q.alpha = a - bb / c;
          q.delta = bb / c;
          q.C = &m.Xn;
          q.fidx = i;
          px.push_back(q);
        }
        E.product(pz);
        E.scratch.reset();
        E.cholesky_inverse(pc);
        E.scratch.reset();
        E.product(py);
        E.scratch.reset();
        E.product(px);
        E.scratch.reset();
        }
        E.fp32 = false;
        E.tol = o.tol;
      }
      if (capture) {
        graph = E.capture_end_launch();
        for (int i : pend) {
          ms[i].inf.graphs += 1;
          ms[i].inf.graph_nodes += graph.nodes;
          ms[i].inf.graph_build_seconds += graph.build_seconds;
        }
      }
      note_peak();
      const std::vector<int> f = E.read_flags(nm);
      graph.release();
      std::vector<int> again;
      for (int i : pend) {
        Member& m = ms[i];
        if (f[i] & 2) {
          set_fail(m, HQ_ERR_NOT_POSDEF, "a leaf of I + c X^T X is not positive definite");
          continue;
        }
        if (f[i] & (8 | 16 | 32)) {
          set_fail(m, HQ_ERR_NONFINITE, (f[i] & 16)   ? "non-finite factors entering a recompression"
                                        : (f[i] & 32) ? "non-finite triangular factor in a recompression"
                                                      : "non-finite singular values in a recompression");
          continue;
        }
        if (f[i] & 4) {
          set_fail(m, HQ_ERR_RANK_OVERFLOW, "stacked factor width above the recompression kernels' limit of 1024");
          continue;
        }
        if (f[i] & 1) {
          bool grown = false;
          for (std::vector<int>* cv : {&m.capX, &m.capZ, &m.capL, &m.capY})
            for (int l = 0; l < m.t.L && l < (int)cv->size(); ++l) {
              const int nc = (int)std::min<int64_t>({(int64_t)(*cv)[l] * 2, (int64_t)o.max_rank, m.t.ldf[l]});
              grown |= nc > (*cv)[l];
              (*cv)[l] = nc;
            }
          if (!grown || attempt > 6) {
            set_fail(m, HQ_ERR_RANK_OVERFLOW, "off-diagonal rank above opts.max_rank");
            continue;
          }
          ++m.inf.redo_count;
          m.pred_miss = true;
          again.push_back(i);
          continue;
        }
        m.X = m.Xn;
      }
      // predicted capacities that overflowed: the repeat also gets at least what X_k's ranks call
      // for (instead of doubling its way up from a far too small prediction)
      if (o.predictor && k >= 1 && !again.empty()) {
        std::vector<const hq::HMat*> xs;
        for (int i : again) xs.push_back(&ms[i].X);
        const std::vector<std::vector<int>> rk = read_ranks_many(E, xs);
        for (size_t j = 0; j < again.size(); ++j) {
          Member& m = ms[again[j]];
          const std::vector<int> g = caps_grow(m.t, rk[j], o.max_rank, 2, 16);
          for (std::vector<int>* cv : {&m.capX, &m.capZ, &m.capL, &m.capY})
            for (int l = 0; l < m.t.L && l < (int)cv->size(); ++l) (*cv)[l] = std::max((*cv)[l], g[l]);
        }
      }
      pend.swap(again);
    }
    cur ^= 1;
    // per-iteration ranks; members whose schedule ends here are finished now, before their
    // iterate's arena is recycled
    std::vector<const hq::HMat*> xs;
    std::vector<int> ok;
    for (int i : act)
      if (ms[i].status == HQ_OK) {
        xs.push_back(&ms[i].X);
        ok.push_back(i);
      }
    if (o.record_ranks && k >= 1)
      for (int i : ok) {
        xs.push_back(&ms[i].Z);
        xs.push_back(&ms[i].Linv);
        xs.push_back(&ms[i].Y);
      }
    const std::vector<std::vector<int>> rk = read_ranks_many(E, xs);
    if (k < 16)
      for (int i : act) ms[i].inf.iter_seconds[k] = secs(tk);
    if (o.record_ranks && k < 16)
      for (size_t j = 0; j < ok.size(); ++j) {
        Member& m = ms[ok[j]];
        for (int q = 0; q < 4; ++q) {
          if (q > 0 && k == 0) break;
          const std::vector<int> lm = level_max(m.t, rk[q == 0 ? j : ok.size() + 3 * j + (q - 1)]);
          for (int l = 0; l < m.t.L && l < 24; ++l) m.inf.level_ranks[k][q][l] = lm[l];
        }
      }
    std::vector<hq::Engine::AffTask> fin;
    pa.reset();
    E.stage.reset();
    E.scratch.reset();
    for (size_t j = 0; j < ok.size(); ++j) {
      Member& m = ms[ok[j]];
      if (k < 16) m.inf.max_rank_iter[k] = max_of(rk[j]);
      if (k + 1 == m.K) {
        // Alg. 3 lines 17-18: U = X_K (symmetrised), P = (I - U)/2
        m.P = E.alloc_hmat_in(pa, &m.t, caps_grow(m.t, rk[j], o.max_rank, 1, 0), false);
        fin.push_back(hq::Engine::AffTask{&m.X, &m.P, projector ? -0.5 : 1.0, projector ? 0.5 : 0.0, ok[j]});
      }
    }
    for (int attempt = 0; !fin.empty(); ++attempt) {
      E.clear_flags(nm);
      E.sym_affine(fin);
      note_peak();
      const std::vector<int> f = E.read_flags(nm);
      std::vector<hq::Engine::AffTask> again;
      for (const auto& a : fin) {
        Member& m = ms[a.fidx];
        if (f[a.fidx] & (8 | 16 | 32)) {
          set_fail(m, HQ_ERR_NONFINITE, "non-finite values in the symmetrisation");
        } else if (f[a.fidx] & 4) {
          set_fail(m, HQ_ERR_RANK_OVERFLOW, "stacked factor width above the recompression kernels' limit of 1024");
        } else if (f[a.fidx] & 1) {  // the symmetric part needs more columns than X_K had
          std::vector<int> cp = m.P.cap;
          bool grown = false;
          for (int l = 0; l < m.t.L; ++l) {
            const int nc = (int)std::min<int64_t>({(int64_t)cp[l] * 2, (int64_t)o.max_rank, m.t.ldf[l]});
            grown |= nc > cp[l];
            cp[l] = nc;
          }
          if (!grown || attempt > 6) {
            set_fail(m, HQ_ERR_RANK_OVERFLOW, "off-diagonal rank above opts.max_rank");
          } else {
            m.P = E.alloc_hmat_in(pa, &m.t, cp, false);
            again.push_back(a);
          }
        }
      }
      for (const auto& a : fin) {
        Member& m = ms[a.fidx];
        if (m.status != HQ_OK || std::any_of(again.begin(), again.end(), [&](const hq::Engine::AffTask& x) {
              return x.fidx == a.fidx;
            }))
          continue;
        m.out = compact_copy(E, m.P, st, o.leaf);
        m.inf.max_rank = m.out ? max_of(E.read_ranks(m.out->H)) : 0;
        m.inf.bytes = (int64_t)m.out->H.bytes();
      }
      E.stage.reset();
      E.scratch.reset();
      fin.swap(again);
    }
  }
  const double total = secs(t0);
  for (Member& m : ms) {
    m.inf.peak_bytes = (int64_t)peak;
    m.inf.launches = E.launches;
    m.inf.seconds = total;
  }
}

// ---- the Zolo-pd driver -----------------------------------------------------------------------
// Zolo-pd (cited in Sec. 2.1; Nakatsukasa and Freund 2016): the setup of Alg. 3 line 1, then the
// steps of zolo_schedule, X <- mhat (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1}):
//   step 0 (X_0 banded): X_0 (X_0^T X_0 + c I)^{-1} = Q1 Q2^T / sqrt(c) with [X_0 / sqrt(c); I] =
//     [Q1; Q2] R, the structured QR of Algorithms 1/2 at scale 1 / (sqrt(c) alpha) (all sweeps of all
//     members on the host in parallel, all products in one batch);
//   steps k >= 1: G = X^T X + c_1 I (one product per member), Z_j = G + (c_{2j-1} - c_1) I sharing
//     G's blocks (only the leaves differ), all H-Cholesky factorisations in one lockstep batch,
//     Y_j = X L_j^{-T} and V_j = Y_j L_j^{-1} (two batched products);
// and X_{k+1} as one HODLR sum of the r + 1 terms per member.  Members of a batch advance together
// (each with its own schedule, degree and status word); capacities come from the previous iterate's
// ranks (twice plus 16) and double for the members that overflow; a member is symmetrised as in
// Alg. 3 as soon as its schedule ends.
void run_zolo(std::vector<Member>& ms, const hq_opts& o, hipStream_t st, bool projector) {
  const auto t0 = clk::now();
  const int nm = (int)ms.size();
  if (nm > hq::Engine::kFlagSlots) throw std::runtime_error("batch larger than the engine's status slots");
  for (Member& m : ms) {
    m.ab.resize((size_t)m.n * m.ldab);
    HQ_CHECK(hipMemcpyAsync(m.ab.data(), m.band, sizeof(double) * m.ab.size(), hipMemcpyDeviceToHost, st));
  }
  HQ_CHECK(hipStreamSynchronize(st));
  std::vector<std::vector<hq::ZoloStep>> zs(nm);
#pragma omp parallel for schedule(dynamic, 1) if (nm > 1)
  for (int i = 0; i < nm; ++i) {
    Member& m = ms[i];
    const auto ts = clk::now();
    std::memset(&m.inf, 0, sizeof(m.inf));
    m.t.build(m.n, o.leaf);
    if (m.t.L > 0 && (int64_t)m.b > m.n / (int64_t(1) << m.t.L)) {
      set_fail(m, HQ_ERR_UNSUPPORTED, "bandwidth exceeds the smallest diagonal block; raise opts.leaf");
      continue;
    }
    m.beff = (int)std::min<int64_t>(m.b, std::max<int64_t>(1, m.n - 1));
    const double alpha = norm_inf_shifted(m.ab.data(), m.n, m.beff, m.ldab, m.mu);
    if (!(alpha > 0.0)) {
      set_fail(m, HQ_ERR_SINGULAR_SHIFT, "A - mu I is zero");
      continue;
    }
    const double dist = certified_distance(m.ab.data(), m.n, m.beff, m.ldab, m.mu, alpha);
    if (!(dist > 0.0)) {
      set_fail(m, HQ_ERR_SINGULAR_SHIFT, "mu is numerically an eigenvalue of A");
      continue;
    }
    zs[i] = hq::zolo_schedule(std::max(dist / alpha, 1e-150), o.delta, o.zolo_r, o.max_iter);
    if (zs[i].empty()) {
      set_fail(m, HQ_ERR_NO_CONVERGENCE, "Zolotarev steps did not reach 1 - delta within max_iter");
      continue;
    }
    m.K = (int)zs[i].size();
    m.inf.alpha = alpha;
    m.inf.l0 = dist / alpha;
    m.inf.iters = m.K;
    m.inf.zolo_r = zs[i][0].r;
    m.inf.levels = m.t.L;
    for (int k = 0; k < m.K && k < 16; ++k) {
      m.inf.a[k] = zs[i][k].mhat;
      m.inf.b[k] = zs[i][k].l;
      m.inf.c[k] = zs[i][k].c[1];
    }
    m.inf.setup_seconds = secs(ts);
  }
  int Kmax = 0;
  for (Member& m : ms)
    if (m.status == HQ_OK) Kmax = std::max(Kmax, m.K);

  hq::Engine E(st);
  E.tol = o.tol;
  hq::DevArena xa[2], it, qa, pa;
  std::unique_ptr<hq::PinnedHost> qimg;
  std::vector<std::vector<hq::HostHodlr>> h1(nm), h2(nm);
  struct Drain {
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{st};
  size_t peak = 0;
  auto note_peak = [&] {
    peak = std::max(peak, E.persist.high_water() + E.scratch.high_water() + E.side_high_water() + xa[0].high_water() +
                              xa[1].high_water() + it.high_water() + qa.high_water() + pa.high_water());
  };
  auto grow = [&](const Member& m, std::vector<int>& cv) {
    bool g = false;
    for (int l = 0; l < m.t.L && l < (int)cv.size(); ++l) {
      const int nc = (int)std::min<int64_t>({(int64_t)cv[l] * 2, (int64_t)o.max_rank, m.t.ldf[l]});
      g |= nc > cv[l];
      cv[l] = nc;
    }
    return g;
  };
  int cur = 0;
  for (Member& m : ms) {
    if (m.status != HQ_OK) continue;
    m.X = E.alloc_hmat_in(xa[cur], &m.t, caps_from(m.t, m.beff, o.max_rank), false);
    build_x0(E, m.band, m.n, m.beff, m.ldab, m.mu, 1.0 / m.inf.alpha, m.X);
  }
  std::vector<std::vector<hq::HMat>> Q1(nm), Q2(nm);
  std::vector<std::vector<int>> capT(nm), capX(nm);  // terms and X_{k+1}, per member
  for (int k = 0; k < Kmax; ++k) {
    std::vector<int> act;
    for (int i = 0; i < nm; ++i)
      if (ms[i].status == HQ_OK && k < ms[i].K) act.push_back(i);
    if (act.empty()) break;
    const auto tk = clk::now();
    if (k == 0) {
      // every member's r structured QR sweeps on the host in one parallel loop, then the copies
      const auto tg = clk::now();
      std::vector<std::pair<int, int>> jobs;
      std::vector<size_t> off(1, 0);
      for (int i : act) {
        const Member& m = ms[i];
        const int r = zs[i][0].r;
        const size_t per = 2 * hq::host_hodlr_doubles(m.t, std::vector<int>(m.t.L, 2 * m.beff), (int)m.t.maxleaf);
        h1[i].assign(r, hq::HostHodlr());
        h2[i].assign(r, hq::HostHodlr());
        for (int j = 0; j < r; ++j) {
          jobs.push_back({i, j});
          off.push_back(off.back() + per);
        }
      }
      qimg.reset(new hq::PinnedHost(sizeof(double) * off.back()));
      // fewer sweeps than threads: each sweep's replays (its inner parallel loops) get a share of the
      // threads, instead of running serially inside a one-thread outer iteration
      const int nthr = omp_get_max_threads(), nj = (int)jobs.size();
      const int outer = std::max(1, std::min(nj, nthr)), inner = std::max(1, nthr / outer);
      const int levels = omp_get_max_active_levels();
      omp_set_max_active_levels(std::max(levels, 2));
#pragma omp parallel for schedule(dynamic, 1) num_threads(outer)
      for (int q = 0; q < nj; ++q) {
        omp_set_num_threads(inner);
        const int i = jobs[q].first, j = jobs[q].second;
        Member& m = ms[i];
        const std::vector<int> capQ(m.t.L, 2 * m.beff);
        hq::q_factors_from_band(m.ab.data(), m.n, m.beff, m.ldab, m.mu,
                                1.0 / (std::sqrt(zs[i][0].c[2 * j + 1]) * m.inf.alpha), m.t, capQ, (int)m.t.maxleaf,
                                h1[i][j], h2[i][j], qimg->as<double>() + off[q]);
      }
      omp_set_max_active_levels(levels);
      HQ_CHECK(hipStreamSynchronize(st));
      for (int i : act) {
        Member& m = ms[i];
        const int r = zs[i][0].r;
        const std::vector<int> capQ(m.t.L, 2 * m.beff);
        Q1[i].resize(r);
        Q2[i].resize(r);
        for (int j = 0; j < r; ++j) {
          Q1[i][j] = E.alloc_hmat_in(qa, &m.t, capQ, false);
          Q2[i][j] = E.alloc_hmat_in(qa, &m.t, capQ, false);
          upload_host(E, h1[i][j], Q1[i][j], false);
          upload_host(E, h2[i][j], Q2[i][j], false);
        }
        m.inf.givens_seconds = secs(tg);
        capT[i] = caps_from(m.t, 3 * m.beff + 8, o.max_rank);
        capX[i] = caps_from(m.t, 2 * (3 * m.beff + 8), o.max_rank);
      }
    } else {
      std::vector<const hq::HMat*> xs;
      for (int i : act) xs.push_back(&ms[i].X);
      const std::vector<std::vector<int>> rk = read_ranks_many(E, xs);
      for (size_t q = 0; q < act.size(); ++q) {
        capT[act[q]] = caps_grow(ms[act[q]].t, rk[q], o.max_rank, 2, 16);
        capX[act[q]] = capT[act[q]];
      }
    }
    std::vector<int> pend = act;
    xa[cur ^ 1].reset();
    for (int attempt = 0; !pend.empty(); ++attempt) {
      E.stage.reset();
      E.scratch.reset();
      it.reset();
      E.clear_flags(nm);
      // per member: the r weighted terms V_j (and, for k >= 1, the Cholesky data)
      std::vector<std::vector<hq::HMat>> V(nm), Li(nm), Lf(nm), Y(nm), Zj(nm);
      std::vector<hq::HMat> G(nm);
      std::vector<hq::Engine::SumTask> sums;
      for (int i : pend) {
        Member& m = ms[i];
        m.Xn = E.alloc_hmat_in(xa[cur ^ 1], &m.t, capX[i], false);
        m.inf.capacity_columns += capacity_columns(m.t, capX[i]);
        V[i].resize(zs[i][k].r);
        for (hq::HMat& v : V[i]) v = E.alloc_hmat_in(it, &m.t, capT[i], false);
      }
      if (k == 0) {
        std::vector<hq::Engine::ProdTask> pv;
        for (int i : pend) {
          const hq::ZoloStep& z = zs[i][k];
          for (int j = 0; j < z.r; ++j) {
            hq::Engine::ProdTask q;
            q.A = E.view(Q1[i][j]);
            q.B = E.view(Q2[i][j], true);
            q.alpha = z.mhat * z.a[j + 1] / std::sqrt(z.c[2 * j + 1]);
            q.C = &V[i][j];
            q.fidx = i;
            pv.push_back(q);
          }
        }
        E.product(pv);
      } else {
        // G = X^T X + c_1 I, then Z_j = G + (c_{2j-1} - c_1) I with their own leaves
        std::vector<hq::Engine::ProdTask> pg;
        for (int i : pend) {
          Member& m = ms[i];
          G[i] = E.alloc_hmat_in(it, &m.t, capT[i], true);
          hq::Engine::ProdTask q;
          q.A = E.view(m.X, true);
          q.B = E.view(m.X);
          q.d_identity = true;
          q.alpha = 1.0;
          q.delta = zs[i][k].c[1];
          q.C = &G[i];
          q.fidx = i;
          pg.push_back(q);
        }
        E.product(pg);
        E.scratch.reset();
        std::vector<hq::LeafAxpy> ax;
        std::vector<hq::Engine::CholTask> pc;
        int maxleaf = 1;
        for (int i : pend) {
          Member& m = ms[i];
          const hq::ZoloStep& z = zs[i][k];
          maxleaf = std::max(maxleaf, (int)m.t.maxleaf);
          Zj[i].assign(z.r, G[i]);
          for (int j = 1; j < z.r; ++j) {
            Zj[i][j].leaves = it.get<double>((size_t)m.t.nleaves * G[i].ldl * G[i].ldl);
            for (int qn = m.t.ninternal; qn < m.t.nnodes; ++qn) {
              const int li = m.t.leaf_index(qn);
              hq::LeafAxpy x{};
              x.out = Zj[i][j].leaf(li); x.ldo = G[i].ldl; x.X = G[i].leaf(li); x.ldx = G[i].ldl;
              x.m = (int)m.t.size(qn); x.alpha = 1.0; x.gamma = z.c[2 * j + 1] - z.c[1];
              ax.push_back(x);
            }
          }
          const int capS = 2 * max_of(capT[i]) + 16;
          const std::vector<int> capW = E.chol_work_caps(m.t, capT[i], capS);
          Li[i].resize(z.r);
          Lf[i].resize(z.r);
          Y[i].resize(z.r);
          for (int j = 0; j < z.r; ++j) {
            Li[i][j] = E.alloc_hmat_in(it, &m.t, capT[i], false);
            Lf[i][j] = E.alloc_hmat_in(it, &m.t, capW, false);
            Y[i][j] = E.alloc_hmat_in(it, &m.t, capT[i], false);
          }
          for (int j = 0; j < z.r; ++j) pc.push_back(hq::Engine::CholTask{&Zj[i][j], &Li[i][j], &Lf[i][j], capS, i});
        }
        if (!ax.empty()) {
          hq::launch_leaf_axpy(E.stage.upload(ax, st), (int)ax.size(), maxleaf, st);
          ++E.launches;
        }
        E.cholesky_inverse(pc);
        E.scratch.reset();
        std::vector<hq::Engine::ProdTask> py, pv;
        for (int i : pend) {
          const hq::ZoloStep& z = zs[i][k];
          for (int j = 0; j < z.r; ++j) {
            hq::Engine::ProdTask a;
            a.A = E.view(ms[i].X);
            a.B = E.view(Li[i][j], true);  // Y_j = X L_j^{-T}
            a.C = &Y[i][j];
            a.fidx = i;
            py.push_back(a);
            hq::Engine::ProdTask b;
            b.A = E.view(Y[i][j]);
            b.B = E.view(Li[i][j]);  // V_j = Y_j L_j^{-1} = X Z_j^{-1}, weighted
            b.alpha = z.mhat * z.a[j + 1];
            b.C = &V[i][j];
            b.fidx = i;
            pv.push_back(b);
          }
        }
        E.product(py);
        E.scratch.reset();
        E.product(pv);
      }
      E.scratch.reset();
      for (int i : pend) {
        hq::Engine::SumTask sm;
        sm.C = &ms[i].Xn;
        sm.fidx = i;
        sm.terms.push_back({zs[i][k].mhat, &ms[i].X});
        for (hq::HMat& v : V[i]) sm.terms.push_back({1.0, &v});
        sums.push_back(std::move(sm));
      }
      E.sum(sums);
      note_peak();
      const std::vector<int> f = E.read_flags(nm);
      std::vector<int> again;
      for (int i : pend) {
        Member& m = ms[i];
        if (f[i] & 2) {
          set_fail(m, HQ_ERR_NOT_POSDEF, "a leaf of X^T X + c I is not positive definite");
        } else if (f[i] & (8 | 16 | 32)) {
          set_fail(m, HQ_ERR_NONFINITE, "non-finite values in a recompression");
        } else if (f[i] & 4) {
          set_fail(m, HQ_ERR_RANK_OVERFLOW, "stacked factor width above the recompression kernels' limit of 1024");
        } else if (f[i] & 1) {
          const bool g1 = grow(m, capT[i]), g2 = grow(m, capX[i]);
          if ((!g1 && !g2) || attempt > 6) {
            set_fail(m, HQ_ERR_RANK_OVERFLOW, "off-diagonal rank above opts.max_rank");
          } else {
            ++m.inf.redo_count;
            again.push_back(i);
          }
        } else {
          m.X = m.Xn;
        }
      }
      pend.swap(again);
    }
    cur ^= 1;
    // ranks of the new iterates; members whose schedule ends here are finished now, before their
    // iterate's arena is recycled
    std::vector<const hq::HMat*> xs;
    std::vector<int> ok;
    for (int i : act)
      if (ms[i].status == HQ_OK) {
        xs.push_back(&ms[i].X);
        ok.push_back(i);
      }
    const std::vector<std::vector<int>> rk = read_ranks_many(E, xs);
    if (k < 16)
      for (int i : act) ms[i].inf.iter_seconds[k] = secs(tk);
    std::vector<hq::Engine::AffTask> fin;
    std::vector<std::vector<int>> capP(nm);
    for (size_t q = 0; q < ok.size(); ++q) {
      Member& m = ms[ok[q]];
      if (k < 16) m.inf.max_rank_iter[k] = max_of(rk[q]);
      if (k + 1 == m.K) {
        capP[ok[q]] = caps_grow(m.t, rk[q], o.max_rank, 1, 0);
        fin.push_back(hq::Engine::AffTask{&m.X, &m.P, projector ? -0.5 : 1.0, projector ? 0.5 : 0.0, ok[q]});
      }
    }
    // Alg. 3 lines 17-18: U = X_K (symmetrised), P = (I - U)/2
    for (int attempt = 0; !fin.empty(); ++attempt) {
      pa.reset();
      E.stage.reset();
      E.scratch.reset();
      for (const auto& a : fin) ms[a.fidx].P = E.alloc_hmat_in(pa, &ms[a.fidx].t, capP[a.fidx], false);
      E.clear_flags(nm);
      E.sym_affine(fin);
      note_peak();
      const std::vector<int> f = E.read_flags(nm);
      std::vector<hq::Engine::AffTask> again;
      for (const auto& a : fin) {
        Member& m = ms[a.fidx];
        if (f[a.fidx] & (8 | 16 | 32)) {
          set_fail(m, HQ_ERR_NONFINITE, "non-finite values in the symmetrisation");
        } else if (f[a.fidx] & 4) {
          set_fail(m, HQ_ERR_RANK_OVERFLOW, "stacked factor width above the recompression kernels' limit of 1024");
        } else if (f[a.fidx] & 1) {
          if (!grow(m, capP[a.fidx]) || attempt > 6)
            set_fail(m, HQ_ERR_RANK_OVERFLOW, "off-diagonal rank above opts.max_rank");
          else
            again.push_back(a);
        }
      }
      // every member that succeeded is copied out before pa is reset for the repeats
      for (const auto& a : fin) {
        Member& m = ms[a.fidx];
        if (m.status != HQ_OK ||
            std::any_of(again.begin(), again.end(), [&](const hq::Engine::AffTask& x) { return x.fidx == a.fidx; }))
          continue;
        m.out = compact_copy(E, m.P, st, o.leaf);
        m.inf.max_rank = m.out ? max_of(E.read_ranks(m.out->H)) : 0;
        m.inf.bytes = (int64_t)m.out->H.bytes();
      }
      fin.swap(again);
    }
  }
  const double total = secs(t0);
  for (Member& m : ms) {
    m.inf.peak_bytes = (int64_t)peak;
    m.inf.launches = E.launches;
    m.inf.seconds = total;
  }
}

hq_status run_qdwh(const double* band, int64_t n, int b, int64_t ldab, double mu, const hq_opts& o, hipStream_t st,
                   bool projector, hq_hodlr_t* out, hq_info* info) {
  std::vector<Member> ms(1);
  ms[0].band = band;
  ms[0].n = n;
  ms[0].b = b;
  ms[0].ldab = ldab;
  ms[0].mu = mu;
  if (o.method == HQ_METHOD_ZOLO)
    run_zolo(ms, o, st, projector);
  else
    run_batch(ms, o, st, projector);
  Member& m = ms[0];
  if (m.status != HQ_OK) {
    if (m.out) hodlr_destroy(m.out);
    return fail(m.status, m.err);
  }
  *out = m.out;
  if (info) *info = m.inf;
  return HQ_OK;
}

}  // namespace

// =============================================================================================
extern "C" {

hq_status hq_default_opts(hq_opts* o) {
  if (!o) return fail(HQ_ERR_ARG, "opts is NULL");
  o->leaf = 256;
  o->tol = 1e-10;
  o->delta = 1e-15;
  o->max_rank = 512;
  o->max_iter = 10;
  o->record_ranks = 0;
  o->predictor = nullptr;
  o->precision = HQ_FP64;
  o->c_fp32_max = 16.0;
  o->graph = 0;
  o->method = HQ_METHOD_QDWH;
  o->zolo_r = 0;
  return HQ_OK;
}

const char* hq_last_error(void) { return g_err.c_str(); }

const char* hq_status_string(hq_status s) {
  switch (s) {
    case HQ_OK: return "ok";
    case HQ_ERR_ARG: return "invalid argument";
    case HQ_ERR_ALLOC: return "allocation failed";
    case HQ_ERR_DEVICE: return "device error";
    case HQ_ERR_UNSUPPORTED: return "unsupported";
    case HQ_ERR_SINGULAR_SHIFT: return "shift is an eigenvalue";
    case HQ_ERR_NOT_POSDEF: return "not positive definite";
    case HQ_ERR_NO_CONVERGENCE: return "no convergence";
    case HQ_ERR_RANK_OVERFLOW: return "rank overflow";
    case HQ_ERR_NONFINITE: return "non-finite values";
  }
  return "unknown status";
}

hq_status hodlr_build(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                      const hq_opts* opts, void* stream, hq_hodlr_t* out) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  hq_opts o;
  hq_status s = check_opts(opts, o);
  if (s) return s;
  if ((s = check_band(band, n, b, ldab))) return s;
  if (!(scale != 0.0)) return fail(HQ_ERR_ARG, "scale must be nonzero");
  return guard([&]() -> hq_status {
    std::unique_ptr<hq_hodlr_s> h(new hq_hodlr_s());
    h->t.build(n, o.leaf);
    if (h->t.L > 0 && (int64_t)b > n / (int64_t(1) << h->t.L))
      return fail(HQ_ERR_UNSUPPORTED, "bandwidth exceeds the smallest diagonal block");
    hipStream_t st = (hipStream_t)stream;
    h->e.reset(new hq::Engine(st));
    h->H = h->e->alloc_hmat(&h->t, caps_from(h->t, b, 1 << 30), false);
    build_x0(*h->e, band, n, b, ldab, shift, 1.0 / scale, h->H);
    HQ_CHECK(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
    h->d_w = h->e->persist.get<int>(1);
    reserve_apply_staging(*h);
    HQ_CHECK(hipEventRecord(h->done, st));
    *out = h.release();
    return HQ_OK;
  });
}

hq_status hodlr_cholesky_solve(hq_hodlr_t H, const double* B, int64_t ldb, int32_t ncols, double* X, int64_t ldx,
                               double tol, int32_t cap, int32_t method, void* stream, double* seconds) {
  if (!H || !B || !X) return fail(HQ_ERR_ARG, "NULL argument");
  const int64_t n = H->t.n;
  if (ncols < 1 || ldb < n || ldx < n) return fail(HQ_ERR_ARG, "bad right-hand side shape");
  if (!(tol > 0.0)) return fail(HQ_ERR_ARG, "tol must be positive");
  if (cap < 0 || cap > hq::kMaxStack) return fail(HQ_ERR_ARG, "cap out of range");
  if (method != 0 && method != 1) return fail(HQ_ERR_ARG, "method must be 0 (substitution) or 1 (inverse)");
  return guard([&]() -> hq_status {
    hipStream_t st = (hipStream_t)stream;
    HQ_CHECK(hipEventSynchronize(H->done));
    hq::Engine E(st);
    E.tol = tol;
    const int c = cap > 0 ? cap : 64;
    const hq::Tree& t = H->t;
    hq::HMat Linv = E.alloc_hmat(&t, caps_from(t, c, 1 << 30), false);
    const std::vector<int> capW = E.chol_work_caps(t, H->H.cap, 2 * c + 16);
    hq::HMat Lf = E.alloc_hmat(&t, capW, false);
    hq::HMat L = E.alloc_hmat(&t, capW, false);
    hq::HMat Zs = H->H;
    Zs.lower_only = true;
    const auto t0 = clk::now();
    E.clear_flags(1);
    E.cholesky_inverse({hq::Engine::CholTask{&Zs, &Linv, &Lf, 2 * c + 16, 0, method == 0 ? &L : nullptr}});
    const int f = E.read_flag();
    if (f & 2) return fail(HQ_ERR_NOT_POSDEF, "a leaf of H is not positive definite");
    if (f & (4 | 8 | 16 | 32)) return fail(HQ_ERR_NONFINITE, "non-finite values in the factorisation");
    if (f & 1) return fail(HQ_ERR_RANK_OVERFLOW, "a block rank above cap");
    const double tf = secs(t0);
    int* dw = E.persist.get<int>(1);
    hq::launch_fill_int(dw, ncols, 1, E.st);
    double* Bw = E.persist.get<double>((size_t)n * ncols);
    double* T1 = E.persist.get<double>((size_t)n * ncols);
    HQ_CHECK(hipMemcpy2DAsync(Bw, sizeof(double) * n, B, sizeof(double) * ldb, sizeof(double) * n, ncols,
                              hipMemcpyDeviceToDevice, E.st));
    HQ_CHECK(hipStreamSynchronize(E.st));
    const auto t1 = clk::now();
    if (method == 0) {
      E.trsm_thin(L, false, Bw, (int)n, T1, (int)n, dw, ncols);  // L T = B (Bw updated in place)
      E.trsm_thin(L, true, T1, (int)n, X, (int)ldx, dw, ncols);  // L^T X = T
    } else {
      E.mm_thin({hq::Engine::ThinTask{E.view(Linv), 0, Bw, (int)n, T1, (int)n, dw, ncols, 1.0, 0.0}});
      E.mm_thin({hq::Engine::ThinTask{E.view(Linv, true), 0, T1, (int)n, X, (int)ldx, dw, ncols, 1.0, 0.0}});
    }
    HQ_CHECK(hipStreamSynchronize(E.st));
    if (seconds) {
      seconds[0] = tf;
      seconds[1] = secs(t1);
    }
    return HQ_OK;
  });
}

hq_status qdwh_sign(const double* band, int64_t n, int32_t b, int64_t ldab, double mu, const hq_opts* opts,
                    void* stream, hq_hodlr_t* sign_out, hq_info* info) {
  if (!sign_out) return fail(HQ_ERR_ARG, "sign_out is NULL");
  *sign_out = nullptr;
  hq_opts o;
  hq_status s = check_opts(opts, o);
  if (s) return s;
  if ((s = check_band(band, n, b, ldab))) return s;
  return guard([&] { return run_qdwh(band, n, b, ldab, mu, o, (hipStream_t)stream, false, sign_out, info); });
}

hq_status spectral_projector(const double* band, int64_t n, int32_t b, int64_t ldab, double mu,
                             const hq_opts* opts, void* stream, hq_hodlr_t* P_out, hq_info* info) {
  if (!P_out) return fail(HQ_ERR_ARG, "P_out is NULL");
  *P_out = nullptr;
  hq_opts o;
  hq_status s = check_opts(opts, o);
  if (s) return s;
  if ((s = check_band(band, n, b, ldab))) return s;
  return guard([&] { return run_qdwh(band, n, b, ldab, mu, o, (hipStream_t)stream, true, P_out, info); });
}

hq_status spectral_projector_batched(int32_t count, const double* const* bands, const int64_t* n, const int32_t* b,
                                     const int64_t* ldab, const double* mu, const hq_opts* opts, void* stream,
                                     hq_hodlr_t* P_out, hq_info* info) {
  if (!P_out) return fail(HQ_ERR_ARG, "P_out is NULL");
  if (count < 1 || count > hq::Engine::kFlagSlots) return fail(HQ_ERR_ARG, "count must be in [1, 1024]");
  for (int i = 0; i < count; ++i) P_out[i] = nullptr;
  if (!bands || !n || !b || !ldab || !mu) return fail(HQ_ERR_ARG, "bands, n, b, ldab or mu is NULL");
  hq_opts o;
  hq_status s = check_opts(opts, o);
  if (s) return s;
  for (int i = 0; i < count; ++i)
    if ((s = check_band(bands[i], n[i], b[i], ldab[i]))) return fail(s, "member " + std::to_string(i) + ": " + g_err);
  return guard([&]() -> hq_status {
    // Members run in consecutive chunks whose estimated working set fits 60% of the free device
    // memory: about 8.5 KB per n (b + 1) L, L the tree depth (measured on banded workloads with
    // capacities of twice the previous ranks).
    const double budget = 0.6 * (double)hq::free_device_bytes();
    std::vector<Member> ms(count);
    for (int i = 0; i < count; ++i) {
      ms[i].band = bands[i];
      ms[i].n = n[i];
      ms[i].b = b[i];
      ms[i].ldab = ldab[i];
      ms[i].mu = mu[i];
    }
    int i0 = 0;
    while (i0 < count) {
      int i1 = i0;
      double sum = 0.0;
      while (i1 < count) {
        hq::Tree t;
        t.build(n[i1], o.leaf);
        // Zolo-pd keeps r Cholesky factorisations and terms per member: about 3.5 times as much
        const double est = (o.method == HQ_METHOD_ZOLO ? 3.5 : 1.0) * 8.5e3 * (double)n[i1] * (b[i1] + 1) *
                               std::max(1, t.L) + 64e6;
        if (i1 > i0 && sum + est > budget) break;
        sum += est;
        ++i1;
      }
      std::vector<Member> chunk(i1 - i0);
      for (int i = i0; i < i1; ++i) {
        chunk[i - i0].band = ms[i].band;
        chunk[i - i0].n = ms[i].n;
        chunk[i - i0].b = ms[i].b;
        chunk[i - i0].ldab = ms[i].ldab;
        chunk[i - i0].mu = ms[i].mu;
      }
      if (o.method == HQ_METHOD_ZOLO)
        run_zolo(chunk, o, (hipStream_t)stream, true);
      else
        run_batch(chunk, o, (hipStream_t)stream, true);
      for (int i = i0; i < i1; ++i) {
        Member& c = chunk[i - i0];
        ms[i].status = c.status;
        ms[i].err = c.err;
        ms[i].inf = c.inf;
        ms[i].out = c.out;
      }
      i0 = i1;
    }
    hq_status first = HQ_OK;
    for (int i = 0; i < count; ++i) {
      Member& m = ms[i];
      if (m.status != HQ_OK) {
        if (m.out) hodlr_destroy(m.out);
        m.out = nullptr;
        if (first == HQ_OK) {
          first = m.status;
          g_err = "member " + std::to_string(i) + ": " + m.err;
        }
      }
      P_out[i] = m.out;
      if (info) info[i] = m.inf;
    }
    return first;
  });
}

hq_status apply_projector(hq_hodlr_t P, const double* X, int64_t ldx, int32_t ncols, double* Y, int64_t ldy,
                          void* stream) {
  if (!P) return fail(HQ_ERR_ARG, "P is NULL");
  if (ncols < 0) return fail(HQ_ERR_ARG, "ncols < 0");
  if (ncols == 0) return HQ_OK;
  if (!X || !Y) return fail(HQ_ERR_ARG, "X or Y is NULL");
  if (ldx < P->t.n || ldy < P->t.n) return fail(HQ_ERR_ARG, "ldx/ldy < n");
  return guard([&]() -> hq_status {
    hq::Engine& e = *P->e;
    HQ_CHECK(hipEventSynchronize(P->done));  // previous call's staging buffers are free again
    e.st = (hipStream_t)stream;
    e.stage.reset();
    e.scratch.reset();
    hq::launch_fill_int(P->d_w, ncols, 1, e.st);
    e.mm_thin({hq::Engine::ThinTask{e.view(P->H), 0, X, (int)ldx, Y, (int)ldy, P->d_w, ncols, 1.0, 0.0}});
    HQ_CHECK(hipEventRecord(P->done, e.st));
    return HQ_OK;
  });
}

hq_status hodlr_to_dense(hq_hodlr_t H, double* out, int64_t ld, void* stream) {
  if (!H || !out) return fail(HQ_ERR_ARG, "NULL argument");
  const int64_t n = H->t.n;
  if (ld < n) return fail(HQ_ERR_ARG, "ld < n");
  return guard([&]() -> hq_status {
    hq::Engine& e = *H->e;
    HQ_CHECK(hipEventSynchronize(H->done));
    e.st = (hipStream_t)stream;
    e.stage.reset();
    e.scratch.reset();
    double* I = e.scratch.get<double>((size_t)n * n);
    std::vector<hq::LeafAxpy> id(1);
    // identity via the leaf kernel over one n x n tile
    id[0] = hq::LeafAxpy{};
    id[0].out = I; id[0].ldo = (int)n; id[0].m = (int)n; id[0].gamma = 1.0; id[0].X = I; id[0].ldx = (int)n;
    hq::launch_leaf_axpy(e.stage.upload(id, e.st), 1, (int)n, e.st);
    hq::launch_fill_int(H->d_w, (int)n, 1, e.st);
    e.mm_thin({hq::Engine::ThinTask{e.view(H->H), 0, I, (int)n, out, (int)ld, H->d_w, (int)n, 1.0, 0.0}});
    HQ_CHECK(hipEventRecord(H->done, e.st));
    HQ_CHECK(hipStreamSynchronize(e.st));
    return HQ_OK;
  });
}

hq_status hodlr_shape(hq_hodlr_t H, int64_t* n, int32_t* levels, int32_t* nleaves, int32_t* max_rank) {
  if (!H) return fail(HQ_ERR_ARG, "H is NULL");
  return guard([&]() -> hq_status {
    if (n) *n = H->t.n;
    if (levels) *levels = H->t.L;
    if (nleaves) *nleaves = H->t.nleaves;
    if (max_rank) {
      HQ_CHECK(hipEventSynchronize(H->done));
      *max_rank = max_of(H->e->read_ranks(H->H));
    }
    return HQ_OK;
  });
}

hq_status hodlr_get_leaf(hq_hodlr_t H, int32_t i, double* out, int64_t ld, int64_t* lo, int64_t* m) {
  if (!H) return fail(HQ_ERR_ARG, "H is NULL");
  if (i < 0 || i >= H->t.nleaves) return fail(HQ_ERR_ARG, "leaf index out of range");
  return guard([&]() -> hq_status {
    const int p = H->t.ninternal + i;
    const int64_t mm = H->t.size(p);
    if (lo) *lo = H->t.lo[p];
    if (m) *m = mm;
    if (out) {
      if (ld < mm) return fail(HQ_ERR_ARG, "ld < m");
      HQ_CHECK(hipEventSynchronize(H->done));
      HQ_CHECK(hipMemcpy2D(out, sizeof(double) * ld, H->H.leaf(i), sizeof(double) * H->H.ldl, sizeof(double) * mm, mm,
                           hipMemcpyDeviceToHost));
    }
    return HQ_OK;
  });
}

hq_status hodlr_get_block(hq_hodlr_t H, int32_t node, int32_t which, double* U, double* V, int64_t ld,
                          int32_t* rank, int64_t* lo, int64_t* mid, int64_t* hi) {
  if (!H) return fail(HQ_ERR_ARG, "H is NULL");
  if (node < 0 || node >= H->t.ninternal) return fail(HQ_ERR_ARG, "node out of range");
  if (which != 0 && which != 1) return fail(HQ_ERR_ARG, "which must be 0 or 1");
  return guard([&]() -> hq_status {
    const hq::Tree& t = H->t;
    if (lo) *lo = t.lo[node];
    if (mid) *mid = t.mid(node);
    if (hi) *hi = t.hi[node];
    HQ_CHECK(hipEventSynchronize(H->done));
    int r = 0;
    HQ_CHECK(hipMemcpy(&r, H->H.rk(node, which), sizeof(int), hipMemcpyDeviceToHost));
    if (rank) *rank = r;
    const int64_t ma = t.size(2 * node + 1), mb = t.size(2 * node + 2);
    const int64_t ru = which == 0 ? ma : mb, rv = which == 0 ? mb : ma;
    if ((U || V) && ld < std::max(ru, rv)) return fail(HQ_ERR_ARG, "ld too small");
    if (U && r > 0)
      HQ_CHECK(hipMemcpy2D(U, sizeof(double) * ld, H->H.U(node, which), sizeof(double) * H->H.ld(node),
                           sizeof(double) * ru, r, hipMemcpyDeviceToHost));
    if (V && r > 0)
      HQ_CHECK(hipMemcpy2D(V, sizeof(double) * ld, H->H.V(node, which), sizeof(double) * H->H.ld(node),
                           sizeof(double) * rv, r, hipMemcpyDeviceToHost));
    return HQ_OK;
  });
}

hq_status hq_shift_for_count(const double* band, int64_t n, int32_t b, int64_t ldab, int64_t nu, double* mu,
                             double* gap) {
  hq_status s = check_band(band, n, b, ldab);
  if (s) return s;
  if (nu < 1 || nu >= n) return fail(HQ_ERR_ARG, "nu must satisfy 1 <= nu < n");
  if (!mu) return fail(HQ_ERR_ARG, "mu is NULL");
  return guard([&]() -> hq_status {
    const double an = norm_inf_shifted(band, n, b, ldab, 0.0);
    const double pm = pivmin_of(band, n, b, ldab);
    double lam[2];
#pragma omp parallel for
    for (int j = 0; j < 2; ++j) {
      std::vector<double> S;
      double lo = -an - 1.0, hi = an + 1.0;
      const int64_t k = nu + j;  // lambda_k, 1-based
      for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (lo + hi);
        if (m <= lo || m >= hi) break;
        if (inertia_below(band, n, b, ldab, m, pm, S) >= k) hi = m;
        else lo = m;
      }
      lam[j] = 0.5 * (lo + hi);
    }
    *mu = 0.5 * (lam[0] + lam[1]);
    if (gap) *gap = lam[1] - lam[0];
    return HQ_OK;
  });
}

void hodlr_destroy(hq_hodlr_t H) {
  if (!H) return;
  if (H->done) (void)hipEventSynchronize(H->done);
  delete H;
}

// ---- test hooks -------------------------------------------------------------------------------
hq_status hq_test_gemm(const double* A, const double* B, double* C, int32_t m, int32_t n, int32_t k, int32_t lda,
                       int32_t ldb, int32_t ldc, int32_t opA, int32_t opB, double alpha, double beta, int32_t fp32,
                       void* stream) {
  if (!A || !B || !C || m < 0 || n < 0 || k < 0) return fail(HQ_ERR_ARG, "bad gemm arguments");
  return guard([&]() -> hq_status {
    hq::Tree t;
    t.build(1, 2);
    hq::Engine e((hipStream_t)stream);
    hq::GemmTask g{};
    g.A = A; g.B = B; g.C = C; g.m = m; g.n = n; g.k = k; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.opA = opA; g.opB = opB; g.alpha = alpha; g.beta = beta;
    e.fp32 = fp32 != 0;
    e.gemm({g}, m, n);
    HQ_CHECK(hipStreamSynchronize(e.st));
    return HQ_OK;
  });
}

hq_status hq_test_qr_r(const double* M, int32_t rows, int32_t r, int32_t ldm, double* R, int32_t fp32,
                       void* stream) {
  if (!M || !R || rows < 1 || r < 1 || ldm < rows) return fail(HQ_ERR_ARG, "bad qr arguments");
  return guard([&]() -> hq_status {
    hq::Tree t;
    t.build(1, 2);
    hq::Engine e((hipStream_t)stream);
    int* dr = e.scratch.get<int>(1);
    hq::launch_fill_int(dr, r, 1, e.st);
    // R-only TSQR with the plan the recompressions use
    const int rc = r;
    const hq::QrPlan pl = hq::plan_qr(rows, rc);
    hq::QrTask q{};
    q.M = M; q.ldm = ldm; q.rows = rows; q.rp = dr; q.rcap = rc; q.R = R; q.ldr = rc;
    q.h0 = pl.h0; q.hs = pl.hs; q.ntiles = pl.ntiles;
    q.work = e.scratch.get<double>((size_t)q.ntiles * q.hs * rc);
    hq::QrTask* dq = e.stage.upload(std::vector<hq::QrTask>{q}, e.st);
    int nst = 0;
    while ((1 << nst) < q.ntiles) ++nst;
    for (int s = 0; s <= nst; ++s)
      hq::launch_qr_stage(dq, 1, s, (q.ntiles + (1 << s) - 1) >> s, e.d_flag, fp32 != 0, e.st);
    HQ_CHECK(hipStreamSynchronize(e.st));
    return HQ_OK;
  });
}

hq_status hq_test_recompress(const double* Us, int32_t m, const double* Vs, int32_t n, int32_t r, double tol,
                             int32_t kcap, double* U, double* V, int32_t* k, int32_t fp32, void* stream) {
  if (!Us || !Vs || !U || !V || !k || m < 1 || n < 1 || r < 0 || kcap < 1) return fail(HQ_ERR_ARG, "bad arguments");
  return guard([&]() -> hq_status {
    hq::Tree t;
    t.build(1, 2);
    hq::Engine e((hipStream_t)stream);
    e.tol = tol;
    int* dr = e.scratch.get<int>(2);
    hq::launch_fill_int(dr, r, 1, e.st);
    hq::Engine::RecTask rt{};
    rt.Us = Us; rt.ldus = m; rt.m = m; rt.Vs = Vs; rt.ldvs = n; rt.n = n; rt.r = dr; rt.rcap = std::max(r, 1);
    rt.U = U; rt.V = V; rt.ldu = m; rt.ldv = n; rt.rank = dr + 1; rt.kcap = kcap; rt.thresh = tol;
    e.fp32 = fp32 != 0;
    e.recompress({rt});
    HQ_CHECK(hipMemcpyAsync(k, dr + 1, sizeof(int), hipMemcpyDeviceToHost, e.st));
    HQ_CHECK(hipStreamSynchronize(e.st));
    const int f = e.read_flag();
    if (f & (8 | 16 | 32)) return fail(HQ_ERR_NONFINITE, "non-finite values in the stacked factors");
    return (f & 1) ? fail(HQ_ERR_RANK_OVERFLOW, "rank above kcap") : HQ_OK;
  });
}

hq_status hq_test_from_dense(const double* dense, int64_t n, int64_t ld, const hq_opts* opts, int32_t cap,
                             void* stream, hq_hodlr_t* out) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  hq_opts o;
  hq_status s = check_opts(opts, o);
  if (s) return s;
  if (!dense || n < 1 || ld < n || cap < 1) return fail(HQ_ERR_ARG, "bad arguments");
  return guard([&]() -> hq_status {
    std::unique_ptr<hq_hodlr_s> h(new hq_hodlr_s());
    h->t.build(n, o.leaf);
    const hq::Tree& t = h->t;
    if (t.L > 0 && t.ldf[0] > 1024) return fail(HQ_ERR_UNSUPPORTED, "test compression limited to n <= 2048");
    hipStream_t st = (hipStream_t)stream;
    h->e.reset(new hq::Engine(st));
    hq::Engine& e = *h->e;
    e.tol = o.tol;
    h->H = e.alloc_hmat(&t, caps_from(t, cap, 1 << 30), false);
    // leaves
    for (int i = 0; i < t.nleaves; ++i) {
      const int p = t.ninternal + i;
      const int64_t lo = t.lo[p], m = t.size(p);
      HQ_CHECK(hipMemcpy2DAsync(h->H.leaf(i), sizeof(double) * h->H.ldl, dense + lo + lo * ld, sizeof(double) * ld,
                                sizeof(double) * m, m, hipMemcpyDeviceToDevice, st));
    }
    // off-diagonal blocks: Us = block (rows x cols), Vs = I (cols x cols)
    std::vector<hq::Engine::RecTask> rec;
    int64_t maxc = 1;
    for (int p = 0; p < t.ninternal; ++p) maxc = std::max(maxc, std::max(t.size(2 * p + 1), t.size(2 * p + 2)));
    double* I = e.scratch.get<double>((size_t)maxc * maxc);
    std::vector<hq::LeafAxpy> id(1);
    id[0] = hq::LeafAxpy{};
    id[0].out = I; id[0].ldo = (int)maxc; id[0].m = (int)maxc; id[0].gamma = 1.0; id[0].X = I; id[0].ldx = (int)maxc;
    hq::launch_leaf_axpy(e.stage.upload(id, st), 1, (int)maxc, st);
    std::vector<int> widths;
    int* dw = e.scratch.get<int>(2 * std::max(1, t.ninternal));
    std::vector<int> hw(2 * std::max(1, t.ninternal));
    for (int p = 0; p < t.ninternal; ++p)
      for (int s2 = 0; s2 < 2; ++s2) {
        const int a = 2 * p + 1, b = 2 * p + 2;
        const int64_t r0 = s2 == 0 ? t.lo[a] : t.lo[b], c0 = s2 == 0 ? t.lo[b] : t.lo[a];
        const int64_t mr = s2 == 0 ? t.size(a) : t.size(b), mc = s2 == 0 ? t.size(b) : t.size(a);
        hw[2 * p + s2] = (int)mc;
        hq::Engine::RecTask rt{};
        rt.Us = dense + r0 + c0 * ld; rt.ldus = (int)ld; rt.m = (int)mr;
        rt.Vs = I; rt.ldvs = (int)maxc; rt.n = (int)mc;
        rt.r = dw + 2 * p + s2; rt.rcap = (int)mc;
        rt.U = h->H.U(p, s2); rt.V = h->H.V(p, s2); rt.ldu = rt.ldv = h->H.ld(p);
        rt.rank = h->H.rk(p, s2); rt.kcap = h->H.capof(p); rt.thresh = o.tol;
        rec.push_back(rt);
      }
    HQ_CHECK(hipMemcpyAsync(dw, hw.data(), sizeof(int) * hw.size(), hipMemcpyHostToDevice, st));
    e.recompress(rec);
    HQ_CHECK(hipStreamSynchronize(st));
    if (e.read_flag() & 1) return fail(HQ_ERR_RANK_OVERFLOW, "rank above cap");
    HQ_CHECK(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
    h->d_w = e.persist.get<int>(1);
    e.stage.reset();
    reserve_apply_staging(*h);
    *out = h.release();
    return HQ_OK;
  });
}

hq_status hq_test_product(hq_hodlr_t A, int32_t transA, hq_hodlr_t B, int32_t transB, double alpha, hq_hodlr_t D,
                          int32_t d_identity, double delta, int32_t lower_only, int32_t cap, double tol, void* stream,
                          hq_hodlr_t* out) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!A || !B) return fail(HQ_ERR_ARG, "A or B is NULL");
  if (A->t.n != B->t.n || A->t.leaf != B->t.leaf) return fail(HQ_ERR_ARG, "A and B differ in structure");
  if (D && (D->t.n != A->t.n || D->t.leaf != A->t.leaf)) return fail(HQ_ERR_ARG, "D differs in structure");
  return guard([&]() -> hq_status {
    hipStream_t st = (hipStream_t)stream;
    HQ_CHECK(hipEventSynchronize(A->done));
    HQ_CHECK(hipEventSynchronize(B->done));
    hq::Engine E(st);
    E.tol = tol;
    hq::HMat C = E.alloc_hmat(&A->t, caps_from(A->t, cap, 1 << 30), lower_only != 0);
    hq::HView dv;
    if (D) dv = E.view(D->H);
    E.product(E.view(A->H, transA != 0), E.view(B->H, transB != 0), D ? &dv : nullptr, d_identity != 0, alpha,
              delta, C);
    if (E.read_flag() & 5) return fail(HQ_ERR_RANK_OVERFLOW, "rank above cap");
    *out = compact_copy(E, C, st, A->t.leaf);
    return HQ_OK;
  });
}

hq_status hq_test_cholesky_inverse(hq_hodlr_t Z, int32_t cap, double tol, void* stream, hq_hodlr_t* out) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!Z) return fail(HQ_ERR_ARG, "Z is NULL");
  return guard([&]() -> hq_status {
    hipStream_t st = (hipStream_t)stream;
    HQ_CHECK(hipEventSynchronize(Z->done));
    hq::Engine E(st);
    E.tol = tol;
    const std::vector<int> c = caps_from(Z->t, cap, 1 << 30);
    hq::HMat Linv = E.alloc_hmat(&Z->t, c, false);
    hq::HMat Lf = E.alloc_hmat(&Z->t, E.chol_work_caps(Z->t, Z->H.cap, 2 * cap + 16), false);
    hq::HMat Zs = Z->H;
    Zs.lower_only = true;
    E.cholesky_inverse(Zs, Linv, Lf, 2 * cap + 16);
    const int f = E.read_flag();
    if (f & 2) return fail(HQ_ERR_NOT_POSDEF, "not positive definite");
    if (f & 5) return fail(HQ_ERR_RANK_OVERFLOW, "rank above cap");
    *out = compact_copy(E, Linv, st, Z->t.leaf);
    return HQ_OK;
  });
}

hq_status hq_test_q_factors(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                            int32_t leaf, void* stream, hq_hodlr_t* q1, hq_hodlr_t* q2, int64_t* nrot) {
  if (!q1 || !q2) return fail(HQ_ERR_ARG, "output NULL");
  *q1 = *q2 = nullptr;
  hq_status s = check_band(band, n, b, ldab);
  if (s) return s;
  if (leaf < 2) return fail(HQ_ERR_ARG, "leaf < 2");
  return guard([&]() -> hq_status {
    hipStream_t st = (hipStream_t)stream;
    hq::Tree t;
    t.build(n, leaf);
    if (t.L > 0 && (int64_t)b > n / (int64_t(1) << t.L)) return fail(HQ_ERR_UNSUPPORTED, "b > smallest leaf");
    const std::vector<int> capQ(t.L, 2 * b);
    hq::HostHodlr h1, h2;
    const int64_t nr = hq::q_factors_from_band(band, n, b, ldab, shift, scale, t, capQ, (int)t.maxleaf, h1, h2);
    if (nrot) *nrot = nr;
    hq::Engine E(st);
    hq::HMat Q1 = E.alloc_hmat(&t, capQ, false), Q2 = E.alloc_hmat(&t, capQ, false);
    upload_host(E, h1, Q1);
    upload_host(E, h2, Q2);
    *q1 = compact_copy(E, Q1, st, leaf);
    *q2 = compact_copy(E, Q2, st, leaf);
    return HQ_OK;
  });
}

hq_status hq_profile_enable(int32_t on) {
  return guard([&]() -> hq_status {
    hq::prof_enable(on != 0);
    return HQ_OK;
  });
}

hq_status hq_profile_select(int32_t mask) {
  return guard([&]() -> hq_status {
    hq::prof_select((unsigned)mask);
    return HQ_OK;
  });
}

hq_status hq_profile_read(hq_kstat* out, int32_t reset) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  return guard([&]() -> hq_status {
    hq::ProfStat st[hq::K_NCLASS];
    hq::prof_read(st, reset != 0);
    for (int c = 0; c < hq::K_NCLASS; ++c) out[c] = hq_kstat{st[c].launches, st[c].ms, st[c].flops, st[c].bytes};
    return HQ_OK;
  });
}

hq_status hq_profile_mfma(double* out, int32_t reset) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  return guard([&]() -> hq_status {
    hq::prof_mfma(out, reset != 0);
    return HQ_OK;
  });
}

hq_status hq_profile_svd(int64_t* out) {
  if (!out) return fail(HQ_ERR_ARG, "out is NULL");
  return guard([&]() -> hq_status {
    unsigned long long v[8];
    hq::prof_svd_stats(v);
    for (int i = 0; i < 8; ++i) out[i] = (int64_t)v[i];
    return HQ_OK;
  });
}

hq_status hq_test_schedule(double l0, double delta, int32_t max_iter, double* a, double* b, double* c, double* l,
                           int32_t* K) {
  return guard([&] {
    if (!(l0 > 0.0) || !(l0 <= 1.0)) return fail(HQ_ERR_ARG, "l0 must lie in (0, 1]");
    if (!(delta > 0.0)) return fail(HQ_ERR_ARG, "delta must be positive");
    if (max_iter < 1 || max_iter > 16) return fail(HQ_ERR_ARG, "max_iter must lie in [1, 16]");
    if (!a || !b || !c || !l || !K) return fail(HQ_ERR_ARG, "output pointer is NULL");
    const Weights w = schedule(l0, delta, max_iter);
    double lk = l0;
    for (size_t k = 0; k < w.a.size(); ++k) {
      a[k] = w.a[k];
      b[k] = w.b[k];
      c[k] = w.c[k];
      l[k] = lk;
      lk = lk * (w.a[k] + w.b[k] * lk * lk) / (1.0 + w.c[k] * lk * lk);
      if (lk > 1.0) lk = 1.0;
    }
    l[w.a.size()] = w.lK;
    *K = (int32_t)w.a.size();
    return HQ_OK;
  });
}

hq_status hodlr_to_hmatrix(hq_hodlr_t P, double tol, void* stream, hq_hmatrix_t* out) {
  if (!P || !out) return fail(HQ_ERR_ARG, "NULL handle or output");
  *out = nullptr;
  if (!(tol > 0.0)) return fail(HQ_ERR_ARG, "tol must be > 0");
  return guard([&]() -> hq_status {
    std::unique_ptr<hq_hmatrix_s> h(new hq_hmatrix_s());
    hipStream_t st = (hipStream_t)stream;
    HQ_CHECK(hipStreamWaitEvent(st, P->done, 0));  // any earlier use of P on its own stream
    try {
      h->H.convert(P->H, tol, st);
    } catch (const std::runtime_error& e) {
      return fail(HQ_ERR_NONFINITE, e.what());
    }
    const std::vector<int> r = P->e->read_ranks(P->H);
    const hq::Tree& t = P->t;
    int64_t b = 0;
    for (int p = 0; p < t.ninternal; ++p) {
      const int64_t sa = t.size(2 * p + 1), sb = t.size(2 * p + 2);
      b += (sa + sb) * (int64_t)(r[2 * p] + r[2 * p + 1]);
    }
    for (int q = t.ninternal; q < t.nnodes; ++q) b += t.size(q) * t.size(q);
    h->hodlr_bytes = 8 * b;
    *out = h.release();
    return HQ_OK;
  });
}

hq_status hmatrix_shape(hq_hmatrix_t H, int64_t* n, int64_t* nlr, int64_t* ndense, int64_t* bytes,
                        int64_t* hodlr_bytes, int32_t* max_rank) {
  if (!H) return fail(HQ_ERR_ARG, "NULL handle");
  if (n) *n = H->H.n;
  if (nlr) *nlr = (int64_t)H->H.lr.size();
  if (ndense) *ndense = (int64_t)H->H.dn.size();
  if (bytes) *bytes = H->H.bytes;
  if (hodlr_bytes) *hodlr_bytes = H->hodlr_bytes;
  if (max_rank) *max_rank = H->H.max_rank;
  return HQ_OK;
}

hq_status hmatrix_get_block(hq_hmatrix_t H, int64_t i, int64_t* row0, int64_t* col0, int64_t* m, int64_t* ncols,
                            int32_t* rank, double* U, double* V, int64_t ld) {
  if (!H || !row0 || !col0 || !m || !ncols || !rank) return fail(HQ_ERR_ARG, "NULL argument");
  const int64_t nlr = (int64_t)H->H.lr.size(), nd = (int64_t)H->H.dn.size();
  if (i < 0 || i >= nlr + nd) return fail(HQ_ERR_ARG, "block index out of range");
  return guard([&]() -> hq_status {
    if (i < nlr) {
      const hq::HMatrixH::LowRank& b = H->H.lr[i];
      const int k = H->H.ranks[i];
      *row0 = b.r0; *col0 = b.c0; *m = b.m; *ncols = b.n; *rank = k;
      if (!U) return HQ_OK;  // sizes only
      if (!V) return fail(HQ_ERR_ARG, "V is NULL for a low-rank block");
      if (ld < std::max(b.m, b.n)) return fail(HQ_ERR_ARG, "ld smaller than the block");
      if (k > 0) {
        HQ_CHECK(hipMemcpy2D(U, sizeof(double) * ld, b.U, sizeof(double) * b.ld, sizeof(double) * b.m, k,
                             hipMemcpyDeviceToHost));
        HQ_CHECK(hipMemcpy2D(V, sizeof(double) * ld, b.V, sizeof(double) * b.ld, sizeof(double) * b.n, k,
                             hipMemcpyDeviceToHost));
      }
    } else {
      const hq::HMatrixH::Dense& d = H->H.dn[i - nlr];
      *row0 = d.r0; *col0 = d.c0; *m = d.m; *ncols = d.n; *rank = -1;
      if (!U) return HQ_OK;  // sizes only
      if (ld < std::max(d.m, d.n)) return fail(HQ_ERR_ARG, "ld smaller than the block");
      const double* src = d.from_leaf ? H->H.leaves + (size_t)d.leaf * H->H.ldl * H->H.ldl : d.D;
      const int64_t lds = d.from_leaf ? H->H.ldl : d.m;
      HQ_CHECK(hipMemcpy2D(U, sizeof(double) * ld, src, sizeof(double) * lds, sizeof(double) * d.m, d.n,
                           hipMemcpyDeviceToHost));
    }
    return HQ_OK;
  });
}

void hmatrix_destroy(hq_hmatrix_t H) { delete H; }

hq_status hq_test_zolo(double l, int32_t r, double* c, double* a, double* mhat, double* lnext) {
  if (!c || !a || !mhat || !lnext) return fail(HQ_ERR_ARG, "NULL output");
  if (!(l >= 1e-150 && l < 1.0) || r < 1 || r > 16) return fail(HQ_ERR_ARG, "l must be in [1e-150, 1), r in [1, 16]");
  return guard([&] {
    const hq::ZoloStep z = hq::zolo_step(l, r);
    for (int i = 0; i <= 2 * r; ++i) c[i] = z.c[i];
    for (int j = 0; j <= r; ++j) a[j] = z.a[j];
    *mhat = z.mhat;
    *lnext = z.lnext;
    return HQ_OK;
  });
}

hq_status hq_test_q_dense_host(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                               int32_t leaf, double* Q1, double* Q2, int64_t* nrot) {
  hq_status s = check_band(band, n, b, ldab);
  if (s) return s;
  if (!Q1 || !Q2 || leaf < 2) return fail(HQ_ERR_ARG, "bad arguments");
  return guard([&]() -> hq_status {
    hq::Tree t;
    t.build(n, leaf);
    if (t.L > 0 && (int64_t)b > n / (int64_t(1) << t.L)) return fail(HQ_ERR_UNSUPPORTED, "b > smallest leaf");
    const std::vector<int> cap(t.L, 2 * b);
    hq::HostHodlr h[2];
    const int ldl = (int)t.maxleaf;
    const int64_t nr = hq::q_factors_from_band(band, n, b, ldab, shift, scale, t, cap, ldl, h[0], h[1]);
    if (nrot) *nrot = nr;
    for (int w = 0; w < 2; ++w) {
      double* Q = w == 0 ? Q1 : Q2;
      std::fill(Q, Q + n * n, 0.0);
      for (int i = 0; i < t.nleaves; ++i) {
        const int p = t.ninternal + i;
        const int64_t lo = t.lo[p], m = t.size(p);
        for (int64_t c = 0; c < m; ++c)
          for (int64_t r = 0; r < m; ++r) Q[(lo + r) + (lo + c) * n] = h[w].leaves[(size_t)i * ldl * ldl + r + c * ldl];
      }
      for (int p = 0; p < t.ninternal; ++p) {
        const int l = hq::Tree::level(p), i = p - ((1 << l) - 1);
        const int64_t ld = t.ldf[l];
        for (int s2 = 0; s2 < 2; ++s2) {
          const int a = 2 * p + 1, bb = 2 * p + 2;
          const int64_t r0 = s2 == 0 ? t.lo[a] : t.lo[bb], c0 = s2 == 0 ? t.lo[bb] : t.lo[a];
          const int64_t mr = s2 == 0 ? t.size(a) : t.size(bb), mc = s2 == 0 ? t.size(bb) : t.size(a);
          const double* U = h[w].U[l] + (size_t)(2 * i + s2) * ld * cap[l];
          const double* V = h[w].V[l] + (size_t)(2 * i + s2) * ld * cap[l];
          const int rk = h[w].rank[2 * p + s2];
          for (int64_t c = 0; c < mc; ++c)
            for (int64_t r = 0; r < mr; ++r) {
              double v = 0.0;
              for (int k = 0; k < rk; ++k) v += U[r + k * ld] * V[c + k * ld];
              Q[(r0 + r) + (c0 + c) * n] = v;
            }
        }
      }
    }
    return HQ_OK;
  });
}

}  // extern "C"

// HODLR engine: storage and formatted arithmetic (Sec. 3.1.1 of the paper, Table complexity_HODLR)
// mapped onto batched kernels.  Work goes to the caller's stream, except what lies off the critical
// path (C blocks of a product, the H-Cholesky's off-diagonal recompressions), which goes to side
// streams joined back through events; sizes that depend on ranks are read by the kernels from
// device memory.
#include "engine.h"

#include <chrono>

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>

namespace hq {

// ---------------------------------------------------------------------------------------------
// Chunk cache.  Every call builds its engine and arenas afresh; the device chunks (256 MiB or one
// larger allocation) and pinned descriptor chunks they release are kept per device for the next
// call instead of going back to the runtime (hipMalloc / hipHostMalloc of large blocks cost
// milliseconds per call, and hipFree synchronises the device).  Chunks are returned only after the
// device has drained, so a later call on any stream may reuse them at once.
namespace {
struct ChunkCache {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<char*>> dev, host;  // (device, capacity) -> chunks
};
ChunkCache& cache() {
  static ChunkCache* c = new ChunkCache;  // never destroyed: chunks live until the process ends
  return *c;
}
int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}
// Smallest cached chunk of capacity in [bytes, 2 bytes], or nullptr.
char* take_cached(std::map<std::pair<int, size_t>, std::vector<char*>>& m, int dev, size_t bytes, size_t& cap) {
  auto it = m.lower_bound({dev, bytes});
  for (; it != m.end() && it->first.first == dev && it->first.second <= 2 * bytes; ++it)
    if (!it->second.empty()) {
      char* p = it->second.back();
      it->second.pop_back();
      cap = it->first.second;
      return p;
    }
  return nullptr;
}
}  // namespace

static char* chunk_alloc(size_t bytes, size_t& cap, bool host) {
  ChunkCache& c = cache();
  const int dev = current_device();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    if (char* p = take_cached(host ? c.host : c.dev, dev, bytes, cap)) return p;
  }
  char* p = nullptr;
  cap = bytes;
  if (host)
    HQ_CHECK(hipHostMalloc((void**)&p, bytes, hipHostMallocDefault));
  else
    HQ_CHECK(hipMalloc((void**)&p, bytes));
  return p;
}
size_t free_device_bytes() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
  ChunkCache& c = cache();
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(c.mu);
  for (const auto& kv : c.dev)
    if (kv.first.first == dev) free_b += kv.first.second * kv.second.size();
  return free_b;
}

static void chunks_release(const std::vector<std::pair<char*, size_t>>& v, bool host) {
  if (v.empty()) return;
  (void)hipDeviceSynchronize();  // no kernel may still use them
  ChunkCache& c = cache();
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(c.mu);
  for (const auto& x : v) (host ? c.host : c.dev)[{dev, x.second}].push_back(x.first);
}

DevArena::~DevArena() {
  if (fixed_) return;  // the caller's buffer
  std::vector<std::pair<char*, size_t>> v;
  for (auto& c : chunks_) v.push_back({c.p, c.cap});
  chunks_release(v, false);
}
void DevArena::attach_fixed(void* p, size_t cap) {
  if (!chunks_.empty()) throw std::logic_error("attach_fixed: the arena already holds chunks");
  chunks_.push_back(Chunk{static_cast<char*>(p), cap, 0});
  cur_ = 0;
  fixed_ = true;
}
void* DevArena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (fixed_) {
    Chunk& c = chunks_[0];
    if (c.used + bytes > c.cap)
      throw NoAlloc("fixed workspace of " + std::to_string(c.cap) + " bytes exhausted (request of " +
                    std::to_string(bytes) + " bytes beyond " + std::to_string(c.used) + " in use)");
    void* p = c.p + c.used;
    c.used += bytes;
    inuse_ += bytes;
    high_ = std::max(high_, inuse_);
    return p;
  }
  while (cur_ < chunks_.size()) {
    Chunk& c = chunks_[cur_];
    if (c.used + bytes <= c.cap) {
      void* p = c.p + c.used;
      c.used += bytes;
      inuse_ += bytes;
      high_ = std::max(high_, inuse_);
      return p;
    }
    ++cur_;
  }
  Chunk c;
  c.p = chunk_alloc(std::max(chunk_bytes, bytes), c.cap, false);
  c.used = bytes;
  chunks_.push_back(c);
  cur_ = chunks_.size() - 1;
  inuse_ += bytes;
  high_ = std::max(high_, inuse_);
  return c.p;
}
void DevArena::rewind(const Mark& m) {
  for (size_t i = m.cur + 1; i < chunks_.size(); ++i) chunks_[i].used = 0;
  if (m.cur < chunks_.size()) chunks_[m.cur].used = m.used;
  cur_ = m.cur;
  inuse_ = m.inuse;
}
void DevArena::reset() {
  for (auto& c : chunks_) c.used = 0;
  cur_ = 0;
  inuse_ = 0;
}

PinnedHost::PinnedHost(size_t bytes) { p_ = chunk_alloc(std::max<size_t>(bytes, 256), cap_, true); }
PinnedHost::~PinnedHost() { chunks_release({{p_, cap_}}, true); }

DescStage::~DescStage() {
  std::vector<std::pair<char*, size_t>> v;
  for (auto& c : chunks_) v.push_back({c.h, c.cap});
  chunks_release(v, true);
}
// Descriptors are written into pinned, device-visible host memory and read by the kernels from
// there: no copy launch per kernel launch (each workgroup reads its few hundred bytes once).  The
// host stores precede the launch that reads them; chunks are reused only after reset(), which the
// callers issue once the stream has drained.
void* DescStage::up(const void* src, size_t bytes, hipStream_t s) {
  (void)s;
  if (bytes == 0) return nullptr;
  const size_t need = (bytes + 255) & ~size_t(255);
  while (cur_ < chunks_.size() && chunks_[cur_].used + need > chunks_[cur_].cap) ++cur_;
  if (cur_ == chunks_.size()) {
    if (no_grow) throw NoAlloc("descriptor staging of " + std::to_string(capacity()) + " bytes exhausted");
    Chunk c;
    c.h = chunk_alloc(std::max(need, size_t(32) << 20), c.cap, true);
    c.used = 0;
    chunks_.push_back(c);
  }
  Chunk& c = chunks_[cur_];
  std::memcpy(c.h + c.used, src, bytes);
  void* d = c.h + c.used;
  c.used += need;
  return d;
}
void DescStage::reset() {
  for (auto& c : chunks_) c.used = 0;
  cur_ = 0;
}
void DescStage::reserve(size_t bytes) {
  for (const auto& c : chunks_)
    if (c.cap >= bytes) return;
  Chunk c;
  c.h = chunk_alloc(std::max(bytes, size_t(32) << 20), c.cap, true);
  c.used = 0;
  chunks_.push_back(c);
}
size_t DescStage::capacity() const {
  size_t b = 0;
  for (const auto& c : chunks_) b += c.cap;
  return b;
}

size_t HMat::bytes() const {
  size_t b = (size_t)t->nleaves * ldl * ldl * sizeof(double);
  for (int l = 0; l < t->L; ++l) b += (size_t)2 * (2 << l) * t->ldf[l] * cap[l] * sizeof(double);
  return b;
}

HView::Blk HView::upper(int p) const {
  const HMat& H = *h;
  if (H.lower_only || trans) return {H.V(p, 1), H.U(p, 1), H.rk(p, 1), H.ld(p), H.capof(p)};
  return {H.U(p, 0), H.V(p, 0), H.rk(p, 0), H.ld(p), H.capof(p)};
}
HView::Blk HView::lower(int p) const {
  const HMat& H = *h;
  if (H.lower_only || !trans) return {H.U(p, 1), H.V(p, 1), H.rk(p, 1), H.ld(p), H.capof(p)};
  return {H.V(p, 0), H.U(p, 0), H.rk(p, 0), H.ld(p), H.capof(p)};
}

// ---------------------------------------------------------------------------------------------
Engine::Engine(hipStream_t s) : st(s) {
  schur_keep = tuning().schur_keep;
  rec_budget = std::max(rec_budget, free_device_bytes() / 4);
  HQ_CHECK(hipMalloc(&d_flag, sizeof(int) * (kFlagSlots + 64)));
  d_zero = d_flag + kFlagSlots;
  HQ_CHECK(hipMemsetAsync(d_flag, 0, sizeof(int) * (kFlagSlots + 64), st));
}
Engine::~Engine() {
  if (capturing) {  // an error inside a capture: end it and drop the partial graph
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
  }
  if (cap_stream) {
    (void)hipStreamSynchronize(cap_stream);
    (void)hipStreamDestroy(cap_stream);
  }
  for (hipStream_t& sd : sides_)
    if (sd) {
      (void)hipStreamSynchronize(sd);
      (void)hipStreamDestroy(sd);
    }
  for (hipEvent_t e : ev_all) (void)hipEventDestroy(e);
  if (d_flag) (void)hipFree(d_flag);
}

hipStream_t Engine::side_stream(int i) {
  hipStream_t& sd = sides_[i % kSides];
  if (!sd) HQ_CHECK(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
  return sd;
}

hipEvent_t Engine::take_event() {
  if (!ev_free.empty()) {
    hipEvent_t e = ev_free.back();
    ev_free.pop_back();
    return e;
  }
  hipEvent_t e;
  HQ_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  ev_all.push_back(e);
  return e;
}

HMat Engine::alloc_hmat_in(DevArena& ar, const Tree* t, const std::vector<int>& cap, bool lower_only) {
  HMat h;
  h.t = t;
  h.cap = cap;
  h.lower_only = lower_only;
  h.ldl = (int)t->maxleaf;
  h.leaves = ar.get<double>((size_t)t->nleaves * h.ldl * h.ldl);
  h.Ubase.resize(t->L);
  h.Vbase.resize(t->L);
  for (int l = 0; l < t->L; ++l) {
    const size_t per = (size_t)(2 << l) * t->ldf[l] * cap[l];
    h.Ubase[l] = ar.get<double>(per);
    h.Vbase[l] = ar.get<double>(per);
  }
  h.rank = ar.get<int>(std::max(1, 2 * t->ninternal));
  zero_ranks(h);
  return h;
}
void Engine::zero_ranks(HMat& h) { launch_fill_int(h.rank, 0, 2 * h.t->ninternal, st); }

// Products whose k is a long true dimension (Gram matrices, V^T X over a block's rows) split K over
// workgroups into a scratch workspace; the split depends on k alone.
void Engine::gemm(const std::vector<GemmTask>& v0, int max_m, int max_n) {
  if (v0.empty()) return;
  std::vector<GemmTask> v = v0;
  const DevArena::Mark mk = scratch.mark();
  int zmax = 1;
  for (GemmTask& g : v) {
    const int S = g.kp ? 1 : gemm_splits(g.k);
    if (S > 1 && g.m > 0 && g.n > 0) {
      const size_t tiles = (size_t)((g.m + 63) / 64) * ((g.n + 63) / 64);
      g.W = scratch.get<double>(tiles * S * 64 * 64);
      g.splits = S;
      zmax = std::max(zmax, S);
    }
  }
  launch_gemm(stage.upload(v, st), (int)v.size(), max_m, max_n, fp32, st, zmax);
  launches += zmax > 1 ? 2 : 1;
  if (!keep_scratch) scratch.rewind(mk);  // later users of this memory are issued after the reduction (stream order)
}
void Engine::stack(const std::vector<StackTask>& v, int max_rows) {
  if (v.empty()) return;
  launch_stack(stage.upload(v, st), (int)v.size(), max_rows, d_flag, st);
  ++launches;
}

std::vector<int> Engine::read_flags(int count) {
  if (count < 1 || count > kFlagSlots) throw std::runtime_error("read_flags: count out of range");
  std::vector<int> f(count, 0);
  HQ_CHECK(hipMemcpyAsync(f.data(), d_flag, sizeof(int) * count, hipMemcpyDeviceToHost, st));
  HQ_CHECK(hipStreamSynchronize(st));
  return f;
}
void Engine::clear_flags(int count) {
  if (count < 1 || count > kFlagSlots) throw std::runtime_error("clear_flags: count out of range");
  launch_fill_int(d_flag, 0, count, st);
}

std::vector<int> Engine::read_ranks(const HMat& h) {
  std::vector<int> r(std::max(1, 2 * h.t->ninternal));
  HQ_CHECK(hipMemcpyAsync(r.data(), h.rank, sizeof(int) * r.size(), hipMemcpyDeviceToHost, st));
  HQ_CHECK(hipStreamSynchronize(st));
  return r;
}

// ---------------------------------------------------------------------------------------------
// HODLR (subtree) x thin dense: leaves, then per internal node V^T X (all at once), then U (V^T X)
// per level so that updates of one launch never overlap.
void Engine::mm_thin(const std::vector<ThinTask>& tasks) {
  if (tasks.empty()) return;
  int Lmax = 0, maxleaf = 1;
  for (const ThinTask& T : tasks) {
    Lmax = std::max(Lmax, T.H.h->t->L);
    maxleaf = std::max(maxleaf, (int)T.H.h->t->maxleaf);
  }
  std::vector<GemmTask> leafv, tv;
  std::vector<std::vector<GemmTask>> upd(Lmax);
  int wmax = 1, capmax = 1;
  int64_t rowmax = 1;
  for (const ThinTask& T : tasks) {
    const Tree* t = T.H.h->t;
    const int L = t->L;
    wmax = std::max(wmax, T.wcap);
    const int lr = Tree::level(T.root);
    const int64_t r0 = t->lo[T.root];
    // leaves
    const int nl = 1 << (L - lr);
    const int first = ((T.root + 1) << (L - lr)) - 1;
    for (int q = first; q < first + nl; ++q) {
      const int64_t off = t->lo[q] - r0, m = t->size(q);
      GemmTask g{};
      g.A = T.H.h->leaf(t->leaf_index(q));
      g.opA = (T.H.trans && !T.H.h->lower_only) ? 1 : 0;
      g.lda = T.H.h->ldl;
      g.B = T.X + off;
      g.ldb = T.ldx;
      g.C = T.Y + off;
      g.ldc = T.ldy;
      g.m = (int)m;
      g.k = (int)m;
      g.n = T.wcap;
      g.np = T.w;
      g.alpha = T.alpha;
      g.beta = T.beta;
      leafv.push_back(g);
    }
    // internal nodes of the subtree
    for (int l = lr; l < L; ++l) {
      const int cnt = 1 << (l - lr);
      const int f0 = ((T.root + 1) << (l - lr)) - 1;
      for (int q = f0; q < f0 + cnt; ++q) {
        const int a = 2 * q + 1, b = 2 * q + 2;
        const int64_t oa = t->lo[a] - r0, ob = t->lo[b] - r0;
        for (int s = 0; s < 2; ++s) {
          const HView::Blk B = s == 0 ? T.H.upper(q) : T.H.lower(q);
          // s = 0: rows a, cols b;  s = 1: rows b, cols a
          const int64_t orow = s == 0 ? oa : ob, ocol = s == 0 ? ob : oa;
          const int64_t mrow = s == 0 ? t->size(a) : t->size(b), mcol = s == 0 ? t->size(b) : t->size(a);
          double* tmp = scratch.get<double>((size_t)B.cap * T.wcap);
          capmax = std::max(capmax, B.cap);
          rowmax = std::max(rowmax, mrow);
          GemmTask g{};
          g.A = B.V;
          g.opA = 1;
          g.lda = B.ld;
          g.B = T.X + ocol;
          g.ldb = T.ldx;
          g.C = tmp;
          g.ldc = B.cap;
          g.m = B.cap;
          g.mp = B.r;
          g.n = T.wcap;
          g.np = T.w;
          g.k = (int)mcol;
          g.alpha = 1.0;
          g.beta = 0.0;
          tv.push_back(g);
          GemmTask u{};
          u.A = B.U;
          u.lda = B.ld;
          u.B = tmp;
          u.ldb = B.cap;
          u.C = T.Y + orow;
          u.ldc = T.ldy;
          u.m = (int)mrow;
          u.n = T.wcap;
          u.np = T.w;
          u.k = B.cap;
          u.kp = B.r;
          u.alpha = T.alpha;
          u.beta = 1.0;
          upd[l].push_back(u);
        }
      }
    }
  }
  gemm(leafv, maxleaf, wmax);
  gemm(tv, capmax, wmax);
  for (int l = 0; l < Lmax; ++l) gemm(upd[l], (int)rowmax, wmax);
}

void Engine::Graph::release() {
  if (x) (void)hipGraphExecDestroy(x);
  if (g) (void)hipGraphDestroy(g);
  x = nullptr;
  g = nullptr;
}
// The capture runs on a stream of the engine's own (the caller's stream may be the null stream,
// which cannot be captured); it starts after the caller's stream's earlier work, and the graph is
// launched on the caller's stream.
void Engine::capture_begin() {
  if (capturing) throw std::logic_error("capture_begin: already capturing");
  if (!cap_stream) HQ_CHECK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  hipEvent_t e = take_event();
  HQ_CHECK(hipEventRecord(e, st));
  HQ_CHECK(hipStreamWaitEvent(cap_stream, e, 0));
  give_event(e);
  cap_t0 = std::chrono::steady_clock::now();
  caller_st = st;
  st = cap_stream;
  capturing = true;
  HQ_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
}
Engine::Graph Engine::capture_end_launch() {
  if (!capturing) throw std::logic_error("capture_end_launch: not capturing");
  capturing = false;
  Graph G;
  const hipError_t e = hipStreamEndCapture(st, &G.g);
  st = caller_st;
  HQ_CHECK(e);
  size_t nn = 0;
  HQ_CHECK(hipGraphGetNodes(G.g, nullptr, &nn));
  G.nodes = (int64_t)nn;
  HQ_CHECK(hipGraphInstantiate(&G.x, G.g, nullptr, nullptr, 0));
  G.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - cap_t0).count();
  HQ_CHECK(hipGraphLaunch(G.x, st));
  return G;
}

size_t Engine::thin_scratch_bytes(const std::vector<ThinTask>& tasks) {
  auto granule = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
  auto splitk = [&](int m, int n, int k) -> size_t {  // Engine::gemm's workspace of one task (kp unset)
    const int S = gemm_splits(k);
    if (S <= 1 || m <= 0 || n <= 0) return 0;
    const size_t tiles = (size_t)((m + 63) / 64) * ((n + 63) / 64);
    return granule(sizeof(double) * tiles * S * 64 * 64);
  };
  size_t tmp = 0, ws_leaf = 0, ws_t = 0;
  for (const ThinTask& T : tasks) {
    const Tree* t = T.H.h->t;
    const int lr = Tree::level(T.root), L = t->L;
    const int nl = 1 << (L - lr), first = ((T.root + 1) << (L - lr)) - 1;
    for (int q = first; q < first + nl; ++q) ws_leaf += splitk((int)t->size(q), T.wcap, (int)t->size(q));
    for (int l = lr; l < L; ++l) {
      const int cnt = 1 << (l - lr), f0 = ((T.root + 1) << (l - lr)) - 1;
      for (int q = f0; q < f0 + cnt; ++q)
        for (int s = 0; s < 2; ++s) {
          const HView::Blk B = s == 0 ? T.H.upper(q) : T.H.lower(q);
          const int64_t mcol = s == 0 ? t->size(2 * q + 2) : t->size(2 * q + 1);
          tmp += granule(sizeof(double) * (size_t)B.cap * T.wcap);
          ws_t += splitk(B.cap, T.wcap, (int)mcol);
        }
    }
  }
  return tmp + std::max(ws_leaf, ws_t);
}

// ---------------------------------------------------------------------------------------------
// R-only TSQR of each stack, SVD of the small core, and two thin GEMMs per factor.
QrPlan plan_qr(int m, int rcap) {
  // Row tiles depend on m alone (never on capacities), so a result does not change when a
  // capacity does; slots hold a tile or two stacked triangles, whichever is taller.
  const int kTile = tuning().qr_tile_rows;
  QrPlan p;
  p.h0 = m <= kTile ? std::max(m, 1) : kTile;
  p.ntiles = (m + p.h0 - 1) / p.h0;
  p.hs = p.ntiles == 1 ? p.h0 : std::max(p.h0, 2 * rcap);
  return p;
}

namespace {
// Device workspace of one recompression task (TSQR slots of both sides, cores, outputs).
// Leading dimension of the core-SVD workspaces: rows padded to a multiple of 32 (the kernel keeps
// whole 16- or 32-row segments of a column in registers).
int svd_ld(int rc) { return (std::max(rc, 1) + 31) & ~31; }

size_t rec_bytes(int m, int n, int rcap, int kcap) {
  const size_t rc = std::max(rcap, 1), kc = std::max(kcap, 1), ls = svd_ld(rcap);
  const QrPlan a = plan_qr(m, (int)rc), b = plan_qr(n, (int)rc);
  return 8 * (2 * rc * rc + 3 * ls * ls + 2 * rc + 2 * ls * kc + 2 * rc * kc +
              ((size_t)a.ntiles * a.hs + (size_t)b.ntiles * b.hs) * rc) + 4096;
}
// Relative size of the noise FP32 products and Householder steps leave in a stack of m rows
// (u32 sqrt(m), with a safety factor of 4): singular values below it are not kept in FP32 mode.
float fp32_floor(int m) { return 4.0f * 5.9604645e-8f * std::sqrt((float)std::max(m, 1)); }

size_t sym_bytes(int m, int rcap, int kcap) {
  (void)m;
  const size_t rc = std::max(rcap, 1), kc = std::max(kcap, 1), ls = svd_ld(rcap);
  return 8 * (3 * ls * ls + 2 * rc + 2 * ls * kc) + 4096;
}
}  // namespace

// Tasks run in groups whose workspace stays under rec_budget; each group's scratch is released
// (stream order keeps the reuse safe) before the next is issued.
void Engine::recompress(const std::vector<RecTask>& tasks) {
  size_t i = 0;
  while (i < tasks.size()) {
    size_t j = i, sum = 0;
    while (j < tasks.size()) {
      const RecTask& T = tasks[j];
      const size_t b = rec_bytes(T.m, T.n, T.rcap, T.kcap);
      if (j > i && sum + b > rec_budget) break;
      sum += b;
      ++j;
    }
    const DevArena::Mark mk = scratch.mark();
    recompress_group(std::vector<RecTask>(tasks.begin() + i, tasks.begin() + j));
    scratch.rewind(mk);
    i = j;
  }
}
void Engine::compress_sym(const std::vector<SymTask>& tasks) {
  size_t i = 0;
  while (i < tasks.size()) {
    size_t j = i, sum = 0;
    while (j < tasks.size()) {
      const size_t b = sym_bytes(tasks[j].m, tasks[j].rcap, tasks[j].kcap);
      if (j > i && sum + b > rec_budget) break;
      sum += b;
      ++j;
    }
    const DevArena::Mark mk = scratch.mark();
    compress_sym_group(std::vector<SymTask>(tasks.begin() + i, tasks.begin() + j));
    scratch.rewind(mk);
    i = j;
  }
}

void Engine::qr_r(const std::vector<QrJob>& jobs) {
  if (jobs.empty()) return;
  std::vector<QrTask> qv;
  int maxtiles = 1;
  for (const QrJob& J : jobs) {
    const int rc = std::max(J.rcap, 1);
    if (rc > kMaxStack) throw std::runtime_error("qr_r: stacked rank capacity above the kernel limit");
    const QrPlan pl = plan_qr(J.rows, rc);
    QrTask q{};
    q.M = J.M; q.ldm = J.ldm; q.rows = J.rows; q.rp = J.r; q.rcap = rc; q.hs = pl.hs; q.h0 = pl.h0;
    q.ntiles = pl.ntiles; q.work = scratch.get<double>((size_t)pl.ntiles * pl.hs * rc); q.R = J.R; q.ldr = rc;
    q.fidx = J.fidx;
    qv.push_back(q);
    maxtiles = std::max(maxtiles, pl.ntiles);
  }
  QrTask* dq = stage.upload(qv, st);
  int nst = 0;
  while ((1 << nst) < maxtiles) ++nst;
  for (int s = 0; s <= nst; ++s) {
    launch_qr_stage(dq, (int)qv.size(), s, (maxtiles + (1 << s) - 1) >> s, d_flag, fp32, st);
    ++launches;
  }
}

void Engine::recompress_group(const std::vector<RecTask>& tasks, hipEvent_t core_after) {
  if (tasks.empty()) return;
  const int nt = (int)tasks.size();
  std::vector<QrTask> qv;
  std::vector<GemmTask> gB, gP, gUV;
  std::vector<SvdTask> sv;
  int maxtiles = 1, hsmax = 1, rmax = 1, kmax = 1, mmax = 1;
  struct Bufs { double *Ru, *Rv, *B, *J, *Jw, *aux, *Wk, *Jk, *Pu, *Pv; };
  std::vector<Bufs> bufs(nt);
  for (int i = 0; i < nt; ++i) {
    const RecTask& T = tasks[i];
    const int rc = std::max(T.rcap, 1);
    if (rc > kMaxStack) throw std::runtime_error("recompress: stacked rank capacity above the kernel limit");
    Bufs& b = bufs[i];
    const size_t rr = (size_t)rc * rc;
    const int ls = svd_ld(rc);
    const size_t ll = (size_t)ls * ls;
    b.Ru = scratch.get<double>(rr);
    b.Rv = T.Rv ? const_cast<double*>(T.Rv) : scratch.get<double>(rr);
    b.B = scratch.get<double>(ll);
    b.J = scratch.get<double>(ll);
    b.Jw = scratch.get<double>(ll);
    b.aux = scratch.get<double>(2 * (size_t)rc);
    b.Wk = scratch.get<double>((size_t)ls * std::max(T.kcap, 1));
    b.Jk = scratch.get<double>((size_t)ls * std::max(T.kcap, 1));
    b.Pu = scratch.get<double>((size_t)rc * std::max(T.kcap, 1));
    b.Pv = scratch.get<double>((size_t)rc * std::max(T.kcap, 1));
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && T.Rv) continue;  // R of Vs given
      const int m = side == 0 ? T.m : T.n;
      const QrPlan pl = plan_qr(m, rc);
      QrTask q{};
      q.M = side == 0 ? T.Us : T.Vs;
      q.ldm = side == 0 ? T.ldus : T.ldvs;
      q.rows = m;
      q.rp = T.r;
      q.rcap = rc;
      q.hs = pl.hs;
      q.h0 = pl.h0;
      q.ntiles = pl.ntiles;
      q.work = scratch.get<double>((size_t)pl.ntiles * pl.hs * rc);
      q.R = side == 0 ? b.Ru : b.Rv;
      q.ldr = rc;
      q.fidx = T.fidx;
      qv.push_back(q);
      maxtiles = std::max(maxtiles, pl.ntiles);
      hsmax = std::max(hsmax, pl.hs);
    }
    rmax = std::max(rmax, rc);
    kmax = std::max(kmax, T.kcap);
    mmax = std::max(mmax, std::max(T.m, T.n));
    GemmTask g{};  // B = Ru Rv^T
    g.A = b.Ru; g.lda = rc; g.B = b.Rv; g.ldb = rc; g.opB = 1; g.C = b.B; g.ldc = ls;
    g.m = g.n = g.k = rc; g.mp = g.np = g.kp = T.r; g.alpha = 1.0; g.beta = 0.0;
    gB.push_back(g);
    SvdTask s{};
    s.B = b.B; s.C = b.J; s.Jw = b.Jw; s.aux = b.aux; s.Wk = b.Wk; s.Jk = b.Jk; s.sig = nullptr; s.rp = T.r;
    s.kout = T.rank; s.ld = ls; s.kcap = T.kcap; s.thresh = T.thresh; s.qr_thresh = 0.1 * T.thresh;
    s.fidx = T.fidx; s.fp32_floor = fp32_floor(std::max(T.m, T.n));
    s.rlim = std::max(T.m, T.n);  // R factors of stacks with fewer rows than columns end in zero rows
    sv.push_back(s);
    GemmTask pu{};  // Pu = Rv^T Jk
    pu.A = b.Rv; pu.opA = 1; pu.lda = rc; pu.B = b.Jk; pu.ldb = ls; pu.C = b.Pu; pu.ldc = rc;
    pu.m = rc; pu.mp = T.r; pu.n = T.kcap; pu.np = T.rank; pu.k = rc; pu.kp = T.r; pu.alpha = 1.0; pu.beta = 0.0;
    gP.push_back(pu);
    GemmTask pv = pu;  // Pv = Ru^T Wk
    pv.A = b.Ru; pv.B = b.Wk; pv.C = b.Pv;
    gP.push_back(pv);
    GemmTask gu{};  // U = Us Pu
    gu.A = T.Us; gu.lda = T.ldus; gu.B = b.Pu; gu.ldb = rc; gu.C = T.U; gu.ldc = T.ldu;
    gu.m = T.m; gu.n = T.kcap; gu.np = T.rank; gu.k = rc; gu.kp = T.r; gu.alpha = 1.0; gu.beta = 0.0;
    gUV.push_back(gu);
    GemmTask gv = gu;  // V = Vs Pv
    gv.A = T.Vs; gv.lda = T.ldvs; gv.B = b.Pv; gv.C = T.V; gv.ldc = T.ldv; gv.m = T.n;
    gUV.push_back(gv);
  }
  QrTask* dq = stage.upload(qv, st);
  int nst = 0;
  while ((1 << nst) < maxtiles) ++nst;
  for (int s = 0; s <= nst; ++s) {
    const int pairs = (maxtiles + (1 << s) - 1) >> s;
    launch_qr_stage(dq, (int)qv.size(), s, pairs, d_flag, fp32, st);
    ++launches;
  }
  if (core_after) HQ_CHECK(hipStreamWaitEvent(st, core_after, 0));
  gemm(gB, rmax, rmax);
  launch_svd(stage.upload(sv, st), nt, d_flag, fp32, st);
  launches += 2;
  gemm(gP, rmax, kmax);
  gemm(gUV, mmax, kmax);
}

// Symmetric compression through the Gram matrix: G = S^T S (one MFMA GEMM), its singular vectors
// Y (= eigenvectors) keep sigma(G) > thresh^2, and S' = S Y_k.  Then
// ||S S^T - S' S'^T|| = ||(I - P_k) G (I - P_k)|| <= thresh^2 + O(u ||G||) whatever the gaps of G,
// which is all the lazy Schur factor needs (its threshold is far above u^(1/2) ||S||).
void Engine::compress_sym_group(const std::vector<SymTask>& tasks) {
  if (tasks.empty()) return;
  const int nt = (int)tasks.size();
  std::vector<GemmTask> gg, go;
  std::vector<SvdTask> sv;
  int rmax = 1, kmax = 1, mmax = 1;
  for (int i = 0; i < nt; ++i) {
    const SymTask& T = tasks[i];
    const int rc = std::max(T.rcap, 1);
    if (rc > kMaxStack) throw std::runtime_error("compress_sym: factor capacity above the kernel limit");
    const int ls = svd_ld(rc);
    double* G = scratch.get<double>((size_t)ls * ls);
    double* J = scratch.get<double>((size_t)ls * ls);
    double* Jw = scratch.get<double>((size_t)ls * ls);
    double* aux = scratch.get<double>(2 * (size_t)rc);
    double* Jk = scratch.get<double>((size_t)ls * std::max(T.kcap, 1));
    GemmTask g{};  // G = S^T S
    g.A = T.S; g.opA = 1; g.lda = T.lds; g.B = T.S; g.ldb = T.lds; g.C = G; g.ldc = ls;
    g.m = g.n = rc; g.mp = g.np = T.r; g.k = T.m; g.alpha = 1.0; g.beta = 0.0;
    gg.push_back(g);
    rmax = std::max(rmax, rc);
    kmax = std::max(kmax, T.kcap);
    mmax = std::max(mmax, T.m);
    SvdTask s{};
    const double th2 = T.thresh * T.thresh;
    // only the right singular vectors (G's eigenvectors) are used: no left ones (Wk null)
    s.B = G; s.C = J; s.Jw = Jw; s.aux = aux; s.Wk = nullptr; s.Jk = Jk; s.rp = T.r; s.kout = T.rank; s.ld = ls;
    s.kcap = T.kcap; s.thresh = th2; s.qr_thresh = 0.1 * th2; s.fidx = T.fidx;
    s.fp32_floor = fp32_floor(T.m);
    s.keep_below = T.keep_below;
    sv.push_back(s);
    GemmTask o{};  // out = S Jk
    o.A = T.S; o.lda = T.lds; o.B = Jk; o.ldb = ls; o.C = T.out; o.ldc = T.ldo;
    o.m = T.m; o.n = T.kcap; o.np = T.rank; o.k = rc; o.kp = T.r; o.alpha = 1.0; o.beta = 0.0;
    go.push_back(o);
  }
  gemm(gg, rmax, rmax);
  launch_svd(stage.upload(sv, st), nt, d_flag, fp32, st);
  ++launches;
  gemm(go, mmax, kmax);
}

// ---------------------------------------------------------------------------------------------
// Formatted product.  For node p with children a, b:
//   C_ab = A_aa B_ab + A_ab B_bb + T_p|ab,   C_ba = A_ba B_aa + A_bb B_ba + T_p|ba,
// where T_p collects the low-rank products that ancestors of p contribute inside p x p:
//   T_a = T_p|aa + A_ab B_ba,   T_b = T_p|bb + A_ba B_ab,
// carried top-down in factored, recompressed form.  Leaves: C_i = A_i B_i + T_i.
// All members of the batch share every launch; a member takes part in level l if its tree has it.
void Engine::product(HView A, HView B, const HView* D, bool d_identity, double alpha, double delta, HMat& C) {
  ProdTask q;
  q.A = A;
  q.B = B;
  if (D) q.D = *D;
  q.d_identity = d_identity;
  q.alpha = alpha;
  q.delta = delta;
  q.C = &C;
  product(std::vector<ProdTask>{q});
}

void Engine::product(const std::vector<ProdTask>& batch) {
  if (batch.empty()) return;
  const double tolT = 0.25 * tol;
  struct NodeBufs {
    double *P1 = nullptr, *P2 = nullptr, *P3 = nullptr, *P4 = nullptr;
    int c1 = 0, c2 = 0, c3 = 0, c4 = 0;
  };
  struct TermF { double* E; double* F; int ld; const int* r; int cap; };
  const int nm = (int)batch.size();
  std::vector<std::vector<NodeBufs>> nbm(nm);
  std::vector<std::vector<TermF>> termm(nm);
  int Lmax = 0;
  // 1) thin products for every internal node of every member
  std::vector<ThinTask> thin;
  for (int m = 0; m < nm; ++m) {
    const ProdTask& P = batch[m];
    const Tree* t = P.C->t;
    const bool full = !P.C->lower_only;
    Lmax = std::max(Lmax, t->L);
    std::vector<NodeBufs>& nb = nbm[m];
    nb.resize(std::max(1, t->ninternal));
    termm[m].assign(t->nnodes, TermF{nullptr, nullptr, 1, d_zero, 0});
    for (int p = 0; p < t->ninternal; ++p) {
      const int a = 2 * p + 1, b = 2 * p + 2, ld = (int)t->ldf[Tree::level(p)];
      const HView::Blk Au = P.A.upper(p), Al = P.A.lower(p), Bu = P.B.upper(p), Bl = P.B.lower(p);
      NodeBufs& q = nb[p];
      if (full) {
        q.c1 = Bu.cap;
        q.P1 = scratch.get<double>((size_t)ld * q.c1);
        thin.push_back({P.A, a, Bu.U, Bu.ld, q.P1, ld, Bu.r, Bu.cap, 1.0, 0.0});  // A_aa Uu_B
        q.c2 = Au.cap;
        q.P2 = scratch.get<double>((size_t)ld * q.c2);
        thin.push_back({P.B.T(), b, Au.V, Au.ld, q.P2, ld, Au.r, Au.cap, 1.0, 0.0});  // B_bb^T Vu_A
      }
      q.c3 = Bl.cap;
      q.P3 = scratch.get<double>((size_t)ld * q.c3);
      thin.push_back({P.A, b, Bl.U, Bl.ld, q.P3, ld, Bl.r, Bl.cap, 1.0, 0.0});  // A_bb Ul_B
      q.c4 = Al.cap;
      q.P4 = scratch.get<double>((size_t)ld * q.c4);
      thin.push_back({P.B.T(), a, Al.V, Al.ld, q.P4, ld, Al.r, Al.cap, 1.0, 0.0});  // B_aa^T Vl_A
    }
  }
  // The thin products only feed the C blocks: they run on side stream 0, ahead of the C blocks of
  // level 0, while the library stream starts on the terms.
  hipEvent_t thin_ready = take_event();
  {
    const hipStream_t sd = side_stream(0);
    hipEvent_t ev = take_event();
    HQ_CHECK(hipEventRecord(ev, st));
    HQ_CHECK(hipStreamWaitEvent(sd, ev, 0));
    give_event(ev);
    const hipStream_t main_st = st;
    st = sd;
    keep_scratch = true;
    try {
      mm_thin(thin);
    } catch (...) {
      st = main_st;
      keep_scratch = false;
      throw;
    }
    st = main_st;
    keep_scratch = false;
    HQ_CHECK(hipEventRecord(thin_ready, sd));
  }

  // 2) level sweep: the accumulated terms of level l+1 (each level needs the previous one's).  The
  // children's terms are allocated first and kept; everything else of the level is released after
  // its launches.
  std::vector<hipEvent_t> cdone;
  for (int l = 0; l < Lmax; ++l) {
    for (int m = 0; m < nm; ++m) {
      const ProdTask& P = batch[m];
      const Tree* t = P.C->t;
      if (l >= t->L) continue;
      const int f0 = (1 << l) - 1, cnt = 1 << l;
      const int ldc = (int)t->ldf[l];
      // terms of leaves only enter the dense leaf products: they stay stacked (no recompression)
      const bool raw = l == t->L - 1;
      for (int p = f0; p < f0 + cnt; ++p) {
        const int64_t sa = t->size(2 * p + 1), sb = t->size(2 * p + 2);
        const HView::Blk Au = P.A.upper(p), Bu = P.B.upper(p), Bl = P.B.lower(p);
        const int capT = std::min<int>({(int)std::max(sa, sb), std::max(P.C->cap[l], std::max(Au.cap, Bu.cap)) * 2, kMaxStack});
        for (int c = 2 * p + 1; c <= 2 * p + 2; ++c) {
          TermF nt;
          nt.ld = ldc;
          nt.cap = raw ? std::min(kMaxStack, termm[m][p].cap + (c == 2 * p + 1 ? Bl.cap : Bu.cap)) : capT;
          nt.E = scratch.get<double>((size_t)nt.ld * nt.cap);
          nt.F = scratch.get<double>((size_t)nt.ld * nt.cap);
          nt.r = scratch.get<int>(1);
          termm[m][c] = nt;
        }
      }
    }
    // C blocks of level l feed no later level: they are stacked and recompressed on side stream
    // l mod kSides as soon as the terms of level l exist, while the library stream goes on with the
    // terms of level l+1.  Their stacks and workspace come from that stream's own arena, whose
    // previous contents only work issued earlier on the same stream used.
    {
      std::vector<StackTask> stk;
      std::vector<RecTask> rec;
      int maxrows = 1;
      DevArena& sa_l = side_arena[l % kSides];
      sa_l.reset();
      scratch.swap(sa_l);
      for (int m = 0; m < nm; ++m) {
        const ProdTask& P = batch[m];
        const Tree* t = P.C->t;
        if (l >= t->L) continue;
        const bool full = !P.C->lower_only;
        const HView* D = P.D.h ? &P.D : nullptr;
        const double alpha = P.alpha, delta = P.delta;
        HMat& C = *P.C;
        std::vector<TermF>& term = termm[m];
        const int f0 = (1 << l) - 1, cnt = 1 << l;
        const int ldc = (int)t->ldf[l];
        for (int p = f0; p < f0 + cnt; ++p) {
          const int a = 2 * p + 1, b = 2 * p + 2;
          const int64_t sa = t->size(a), sb = t->size(b), ofa = t->lo[a] - t->lo[p], ofb = t->lo[b] - t->lo[p];
          maxrows = std::max<int>(maxrows, (int)std::max(sa, sb));
          const HView::Blk Au = P.A.upper(p), Al = P.A.lower(p), Bu = P.B.upper(p), Bl = P.B.lower(p);
          const TermF Tp = term[p];
          for (int s = 0; s < 2; ++s) {
            if (s == 0 && !full) continue;
            const int64_t mr = s == 0 ? sa : sb, mc = s == 0 ? sb : sa;
            const int64_t ofr = s == 0 ? ofa : ofb, ofc = s == 0 ? ofb : ofa;
            const HView::Blk Ax = s == 0 ? Au : Al, Bx = s == 0 ? Bu : Bl;
            const NodeBufs& q = nbm[m][p];
            double* P_left = s == 0 ? q.P1 : q.P3;   // A_xx U_B  (rows r)
            double* P_right = s == 0 ? q.P2 : q.P4;  // B_yy^T V_A (rows c)
            HView::Blk Dx{nullptr, nullptr, d_zero, 1, 0};
            if (D && !P.d_identity) Dx = s == 0 ? D->upper(p) : D->lower(p);
            const int rcap = std::min(kMaxStack, Bx.cap + Ax.cap + Tp.cap + Dx.cap);  // wider: flagged by k_stack
            double* Us = scratch.get<double>((size_t)ldc * rcap);
            double* Vs = scratch.get<double>((size_t)ldc * rcap);
            int* rs = scratch.get<int>(1);
            StackTask su{};
            su.dst = Us; su.ld = ldc; su.rows = (int)mr; su.wcap = rcap; su.wout = rs; su.nsrc = 4; su.fidx = P.fidx;
            su.src[0] = {P_left, Bx.r, ldc, Bx.cap, alpha};
            su.src[1] = {Ax.U, Ax.r, Ax.ld, Ax.cap, alpha};
            su.src[2] = {Tp.E ? Tp.E + ofr : nullptr, Tp.r, Tp.ld, Tp.cap, alpha};
            su.src[3] = {Dx.U, Dx.r, Dx.ld, Dx.cap, delta};
            StackTask sv = su;
            sv.dst = Vs; sv.rows = (int)mc; sv.wout = nullptr;
            sv.src[0] = {Bx.V, Bx.r, Bx.ld, Bx.cap, 1.0};
            sv.src[1] = {P_right, Ax.r, ldc, Ax.cap, 1.0};
            sv.src[2] = {Tp.F ? Tp.F + ofc : nullptr, Tp.r, Tp.ld, Tp.cap, 1.0};
            sv.src[3] = {Dx.V, Dx.r, Dx.ld, Dx.cap, 1.0};
            stk.push_back(su);
            stk.push_back(sv);
            RecTask r{};
            r.Us = Us; r.ldus = ldc; r.m = (int)mr; r.Vs = Vs; r.ldvs = ldc; r.n = (int)mc; r.r = rs; r.rcap = rcap;
            r.U = C.U(p, s); r.V = C.V(p, s); r.ldu = r.ldv = ldc; r.rank = C.rk(p, s); r.kcap = C.cap[l];
            r.thresh = tol; r.fidx = P.fidx;
            rec.push_back(r);
          }
        }
      }
      if (!rec.empty()) {
        const hipStream_t sd = side_stream(l);
        hipEvent_t ready = take_event();
        HQ_CHECK(hipEventRecord(ready, st));
        HQ_CHECK(hipStreamWaitEvent(sd, ready, 0));
        HQ_CHECK(hipStreamWaitEvent(sd, thin_ready, 0));
        give_event(ready);
        const hipStream_t main_st = st;
        st = sd;
        keep_scratch = true;
        try {
          stack(stk, maxrows);
          recompress_group(rec);
        } catch (...) {
          scratch.swap(sa_l);
          st = main_st;
          keep_scratch = false;
          throw;
        }
        st = main_st;
        keep_scratch = false;
        hipEvent_t d = take_event();
        HQ_CHECK(hipEventRecord(d, sd));
        cdone.push_back(d);
      }
      scratch.swap(sa_l);
    }
    const DevArena::Mark level_mark = scratch.mark();
    std::vector<GemmTask> gm, gg;
    std::vector<StackTask> stk;
    std::vector<RecTask> rec;
    int maxrows = 1, mcapA = 1, mcapB = 1;
    for (int m = 0; m < nm; ++m) {
      const ProdTask& P = batch[m];
      const Tree* t = P.C->t;
      if (l >= t->L) continue;
      std::vector<TermF>& term = termm[m];
      const int f0 = (1 << l) - 1, cnt = 1 << l;
      const int ldc = (int)t->ldf[l];
      for (int p = f0; p < f0 + cnt; ++p) {
        const int a = 2 * p + 1, b = 2 * p + 2;
        const int64_t sa = t->size(a), sb = t->size(b), ofa = t->lo[a] - t->lo[p], ofb = t->lo[b] - t->lo[p];
        maxrows = std::max<int>(maxrows, (int)std::max(sa, sb));
        const HView::Blk Au = P.A.upper(p), Al = P.A.lower(p), Bu = P.B.upper(p), Bl = P.B.lower(p);
        const TermF Tp = term[p];
        mcapA = std::max(mcapA, std::max(Au.cap, Al.cap));
        mcapB = std::max(mcapB, std::max(Bu.cap, Bl.cap));
        // --- terms for the children: T_a = T_p|aa + Uu_A (Vu_A^T Ul_B) Vl_B^T, T_b = T_p|bb + Ul_A (Vl_A^T Uu_B) Vu_B^T
        for (int s = 0; s < 2; ++s) {
          const int c = s == 0 ? a : b;
          const int64_t mrow = s == 0 ? sa : sb, inner = s == 0 ? sb : sa, ofc = s == 0 ? ofa : ofb;
          const HView::Blk Ax = s == 0 ? Au : Al, By = s == 0 ? Bl : Bu;
          double* M = scratch.get<double>((size_t)std::max(Ax.cap, 1) * std::max(By.cap, 1));
          double* G = scratch.get<double>((size_t)ldc * std::max(By.cap, 1));
          GemmTask g1{};
          g1.A = Ax.V; g1.opA = 1; g1.lda = Ax.ld; g1.B = By.U; g1.ldb = By.ld; g1.C = M; g1.ldc = std::max(Ax.cap, 1);
          g1.m = Ax.cap; g1.mp = Ax.r; g1.n = By.cap; g1.np = By.r; g1.k = (int)inner; g1.alpha = 1.0; g1.beta = 0.0;
          gm.push_back(g1);
          GemmTask g2{};
          g2.A = Ax.U; g2.lda = Ax.ld; g2.B = M; g2.ldb = std::max(Ax.cap, 1); g2.C = G; g2.ldc = ldc;
          g2.m = (int)mrow; g2.n = By.cap; g2.np = By.r; g2.k = Ax.cap; g2.kp = Ax.r; g2.alpha = 1.0; g2.beta = 0.0;
          gg.push_back(g2);
          const int rcap = std::min(kMaxStack, Tp.cap + By.cap);
          const TermF& nt = term[c];
          const bool raw = l == t->L - 1;  // stacked straight into the leaf's term
          double* Us = raw ? nt.E : scratch.get<double>((size_t)ldc * rcap);
          double* Vs = raw ? nt.F : scratch.get<double>((size_t)ldc * rcap);
          int* rs = raw ? const_cast<int*>(nt.r) : scratch.get<int>(1);
          StackTask su{};
          su.dst = Us; su.ld = ldc; su.rows = (int)mrow; su.wcap = rcap; su.wout = rs; su.nsrc = 2; su.fidx = P.fidx;
          su.src[0] = {Tp.E ? Tp.E + ofc : nullptr, Tp.r, Tp.ld, Tp.cap, 1.0};
          su.src[1] = {G, By.r, ldc, By.cap, 1.0};
          StackTask sv = su;
          sv.dst = Vs; sv.wout = nullptr;
          sv.src[0] = {Tp.F ? Tp.F + ofc : nullptr, Tp.r, Tp.ld, Tp.cap, 1.0};
          sv.src[1] = {By.V, By.r, By.ld, By.cap, 1.0};
          stk.push_back(su);
          stk.push_back(sv);
          if (raw) continue;
          RecTask r{};
          r.Us = Us; r.ldus = ldc; r.m = (int)mrow; r.Vs = Vs; r.ldvs = ldc; r.n = (int)mrow; r.r = rs; r.rcap = rcap;
          r.U = nt.E; r.V = nt.F; r.ldu = r.ldv = nt.ld; r.rank = const_cast<int*>(nt.r); r.kcap = nt.cap; r.thresh = tolT;
          r.fidx = P.fidx;
          rec.push_back(r);
        }
      }
    }
    gemm(gm, mcapA, mcapB);
    gemm(gg, maxrows, mcapB);
    stack(stk, maxrows);
    recompress(rec);
    scratch.rewind(level_mark);
  }
  // 3) leaves
  std::vector<GemmTask> g1, g2;
  std::vector<LeafAxpy> ax;
  std::vector<IntCopy> zr;
  int ldlmax = 1;
  for (int m = 0; m < nm; ++m) {
    const ProdTask& P = batch[m];
    const Tree* t = P.C->t;
    const HView* D = P.D.h ? &P.D : nullptr;
    HMat& C = *P.C;
    const int ldl = (int)t->maxleaf;
    ldlmax = std::max(ldlmax, ldl);
    double* tmp = scratch.get<double>((size_t)t->nleaves * ldl * ldl);
    for (int q = t->ninternal; q < t->nnodes; ++q) {
      const int li = t->leaf_index(q), mq = (int)t->size(q);
      double* Ti = tmp + (size_t)li * ldl * ldl;
      GemmTask g{};
      g.A = P.A.h->leaf(li); g.opA = (P.A.trans && !P.A.h->lower_only) ? 1 : 0; g.lda = P.A.h->ldl;
      g.B = P.B.h->leaf(li); g.opB = (P.B.trans && !P.B.h->lower_only) ? 1 : 0; g.ldb = P.B.h->ldl;
      g.C = Ti; g.ldc = ldl; g.m = g.n = g.k = mq; g.alpha = 1.0; g.beta = 0.0;
      g1.push_back(g);
      const TermF& Tq = termm[m][q];
      if (Tq.E) {
        GemmTask e{};
        e.A = Tq.E; e.lda = Tq.ld; e.B = Tq.F; e.ldb = Tq.ld; e.opB = 1; e.C = Ti; e.ldc = ldl;
        e.m = e.n = mq; e.k = Tq.cap; e.kp = Tq.r; e.alpha = 1.0; e.beta = 1.0;
        g2.push_back(e);
      }
      LeafAxpy x{};
      x.out = C.leaf(li); x.ldo = C.ldl; x.m = mq; x.X = Ti; x.ldx = ldl;
      if (C.lower_only) {
        x.Y = Ti; x.ldy = ldl; x.transY = 1; x.alpha = 0.5 * P.alpha; x.beta = 0.5 * P.alpha;
        x.gamma = P.d_identity ? P.delta : 0.0;
      } else {
        x.alpha = P.alpha;
        if (P.d_identity) {
          x.gamma = P.delta;
        } else if (D) {
          x.Y = D->h->leaf(li); x.ldy = D->h->ldl; x.transY = (D->trans && !D->h->lower_only) ? 1 : 0; x.beta = P.delta;
        }
      }
      ax.push_back(x);
    }
    if (C.lower_only)  // lower_only result: upper blocks are implied, keep their ranks at zero
      for (int p = 0; p < t->ninternal; ++p) zr.push_back(IntCopy{C.rk(p, 0), d_zero});
  }
  gemm(g1, ldlmax, ldlmax);
  gemm(g2, ldlmax, ldlmax);
  launch_leaf_axpy(stage.upload(ax, st), (int)ax.size(), ldlmax, st);
  ++launches;
  if (!zr.empty()) {
    launch_copy_ints(stage.upload(zr, st), (int)zr.size(), st);
    ++launches;
  }
  for (hipEvent_t d : cdone) {  // C blocks of every level
    HQ_CHECK(hipStreamWaitEvent(st, d, 0));
    give_event(d);
  }
  HQ_CHECK(hipStreamWaitEvent(st, thin_ready, 0));
  give_event(thin_ready);
}

// ---------------------------------------------------------------------------------------------
// Cholesky and inverse of dense diagonal blocks (A = L L^T in place, X = L^{-1}, X zero on entry), all
// blocks of a list together.  Blocks of at most 128 rows go to the fused register kernel; larger ones
// are split 2 x 2 around h1 = ceil(m / 2):
//   X11 = L11^{-1} (recursively);  L21 = A21 X11^T;  A22 -= L21 L21^T;  X22 = L22^{-1} (recursively);
//   X21 = -X22 (L21 X11),
// with L21 kept in X21's place until the last step.  Every step is one batched launch for all the
// blocks at that depth; FP64 in every precision mode.
void Engine::leaf_chol_inv(const std::vector<LeafTask>& blocks) {
  std::vector<LeafTask> small, big;
  int maxsmall = 1;
  for (const LeafTask& b : blocks) {
    if (b.m <= 0) continue;
    if (b.m <= 128) {
      small.push_back(b);
      maxsmall = std::max(maxsmall, b.m);
    } else {
      big.push_back(b);
    }
  }
  if (!small.empty()) {
    launch_chol_inv(stage.upload(small, st), (int)small.size(), maxsmall, d_flag, st);
    ++launches;
  }
  if (big.empty()) return;
  std::vector<LeafTask> top, bottom;
  std::vector<GemmTask> m1, m2, m3, m4;
  int maxh = 1;
  const DevArena::Mark mk = scratch.mark();
  for (const LeafTask& b : big) {
    const int h1 = (b.m + 1) / 2, h2 = b.m - h1;
    maxh = std::max(maxh, h1);
    double* A = b.A;
    double* X = b.B;
    const int ld = b.lda, ldx = b.ldb;
    double* W = scratch.get<double>((size_t)h2 * h1);
    top.push_back(LeafTask{A, X, h1, ld, ldx, b.fidx});
    bottom.push_back(LeafTask{A + h1 + (size_t)h1 * ld, X + h1 + (size_t)h1 * ldx, h2, ld, ldx, b.fidx});
    GemmTask g{};
    g.A = A + h1; g.lda = ld; g.B = X; g.ldb = ldx; g.opB = 1; g.C = X + h1; g.ldc = ldx;
    g.m = h2; g.n = h1; g.k = h1; g.alpha = 1.0; g.beta = 0.0;
    m1.push_back(g);  // L21 = A21 X11^T
    g = GemmTask{};
    g.A = X + h1; g.lda = ldx; g.B = X + h1; g.ldb = ldx; g.opB = 1; g.C = A + h1 + (size_t)h1 * ld; g.ldc = ld;
    g.m = h2; g.n = h2; g.k = h1; g.alpha = -1.0; g.beta = 1.0;
    m2.push_back(g);  // A22 -= L21 L21^T
    g = GemmTask{};
    g.A = X + h1; g.lda = ldx; g.B = X; g.ldb = ldx; g.C = W; g.ldc = h2;
    g.m = h2; g.n = h1; g.k = h1; g.alpha = 1.0; g.beta = 0.0;
    m3.push_back(g);  // W = L21 X11
    g = GemmTask{};
    g.A = X + h1 + (size_t)h1 * ldx; g.lda = ldx; g.B = W; g.ldb = h2; g.C = X + h1; g.ldc = ldx;
    g.m = h2; g.n = h1; g.k = h2; g.alpha = -1.0; g.beta = 0.0;
    m4.push_back(g);  // X21 = -X22 W
  }
  // the leaf factorisation stays FP64 in every mode
  const bool f = fp32;
  fp32 = false;
  leaf_chol_inv(top);
  gemm(m1, maxh, maxh);
  gemm(m2, maxh, maxh);
  leaf_chol_inv(bottom);
  gemm(m3, maxh, maxh);
  gemm(m4, maxh, maxh);
  fp32 = f;
  scratch.rewind(mk);
}

// ---------------------------------------------------------------------------------------------
// Recursive Cholesky (left subtree, off-diagonal factor, Schur update, right subtree).  The
// Schur complement updates from all ancestors are carried lazily as one symmetric low-rank
// factor S (Z_bb - L_ba L_ba^T restricted = Z_bb - S S^T), compressed at a right turn once it is
// wider than schur_keep columns.  Alongside, the inverse factor is assembled bottom-up:
//   [L^-1]_aa = L_aa^-1, [L^-1]_bb = L_bb^-1, [L^-1]_ba = -(L_bb^-1 U)(L_aa^-T V)^T for L_ba = U V^T.
// A batch runs the recursions of all members in lockstep: a step handles the members' nodes at
// the same position of the depth-first order together, leaves and internal nodes alike.
void Engine::cholesky_inverse(const std::vector<CholTask>& batch) {
  if (batch.empty()) return;
  struct SF { double* p; int ld; const int* r; int cap; };
  struct Item { int m; int c; SF S; };
  const double thS = std::sqrt(0.1 * tol);
  // The inverse during the recursion: Linv's leaves with Lf's off-diagonal blocks, which hold the
  // inverse blocks untruncated (widths of the stacked factors); they are recompressed into Linv's
  // blocks once the recursion is done.
  std::vector<HMat> lw(batch.size());
  for (size_t m = 0; m < batch.size(); ++m) {
    const CholTask& T = batch[m];
    zero_ranks(*T.Linv);
    zero_ranks(*T.Lf);
    if (T.L) {
      zero_ranks(*T.L);
      T.L->leaves = T.Linv->leaves;
      T.L->ldl = T.Linv->ldl;
    }
    lw[m] = *T.Lf;
    lw[m].leaves = T.Linv->leaves;
    lw[m].ldl = T.Linv->ldl;
  }
  std::function<void(const std::vector<Item>&)> dfs = [&](const std::vector<Item>& items) {
    // leaves: Lf_i = chol(Z_i - S S^T), Linv_i = Lf_i^{-1}
    std::vector<LeafAxpy> cp;
    std::vector<GemmTask> gs;
    std::vector<LeafTask> blocks;
    std::vector<Item> inner;
    int maxm = 1;
    for (const Item& it : items) {
      const CholTask& T = batch[it.m];
      const Tree* t = T.Z->t;
      if (!t->is_leaf(it.c)) {
        inner.push_back(it);
        continue;
      }
      const int li = t->leaf_index(it.c), m = (int)t->size(it.c);
      maxm = std::max(maxm, m);
      // A leaf of up to 128 rows is factored by one kernel that only reads its input and writes
      // all of Linv_i: Z_i - S S^T goes straight from Z_i into Lf's leaf (or Z_i itself is the
      // input without a Schur factor).  Larger leaves are factored in place by the 2x2 split, which
      // writes Linv_i's lower part block by block: a copy of Z_i and a zeroed Linv_i first.
      const bool split = m > 128;
      if (split) {
        LeafAxpy x{};
        x.out = T.Lf->leaf(li); x.ldo = T.Lf->ldl; x.X = T.Z->leaf(li); x.ldx = T.Z->ldl; x.m = m; x.alpha = 1.0;
        cp.push_back(x);
        LeafAxpy z{};
        z.out = T.Linv->leaf(li); z.ldo = T.Linv->ldl; z.X = z.out; z.ldx = z.ldo; z.m = m;
        cp.push_back(z);
      }
      const bool schur = it.S.cap > 0;
      if (schur) {
        GemmTask g{};
        g.A = it.S.p; g.lda = it.S.ld; g.B = it.S.p; g.ldb = it.S.ld; g.opB = 1; g.C = T.Lf->leaf(li); g.ldc = T.Lf->ldl;
        g.m = g.n = m; g.k = it.S.cap; g.kp = it.S.r; g.alpha = -1.0; g.beta = 1.0;
        if (!split) {
          g.Cin = T.Z->leaf(li);
          g.ldcin = T.Z->ldl;
        }
        gs.push_back(g);
      }
      if (split || schur)
        blocks.push_back(LeafTask{T.Lf->leaf(li), T.Linv->leaf(li), m, T.Lf->ldl, T.Linv->ldl, T.fidx});
      else
        blocks.push_back(LeafTask{T.Z->leaf(li), T.Linv->leaf(li), m, T.Z->ldl, T.Linv->ldl, T.fidx});
    }
    if (!blocks.empty()) {
      if (!cp.empty()) {
        launch_leaf_axpy(stage.upload(cp, st), (int)cp.size(), maxm, st);
        ++launches;
      }
      gemm(gs, maxm, maxm);
      leaf_chol_inv(blocks);
    }
    if (inner.empty()) return;
    // left subtrees
    std::vector<Item> left;
    for (const Item& it : inner) {
      const Tree* t = batch[it.m].Z->t;
      const int a = 2 * it.c + 1;
      const int64_t la = t->lo[a] - t->lo[it.c];
      left.push_back(Item{it.m, a, SF{it.S.p ? it.S.p + la : nullptr, it.S.ld, it.S.r, it.S.cap}});
    }
    dfs(left);
    // Off-diagonal factor L_ba = (Z_ba - S_b S_a^T) L_aa^{-T} = Us Vs^T with Us = [U(Z_ba), S_b] and
    // Vs = L_aa^{-1} [V(Z_ba), -S_a], and the Schur factor of the right child:
    //   S_b S_b^T + L_ba L_ba^T = Us M Us^T,  M = Vs^T Vs + diag(0 on U(Z_ba)'s columns, I on S_b's),
    // so the new factor is Us C with M = C C^T, the Cholesky factor of the small M, from one Gram
    // GEMM over Vs's rows: no factorisation of the tall Vs on the depth-first chain.  M is positive
    // definite: x^T M x = |Vs x|^2 + |x_S|^2 vanishes only if x_S = 0 and L_aa^{-1} V(Z_ba) x_Z = 0,
    // i.e. x = 0 (V(Z_ba) has orthonormal columns), and its condition is moderate (L_aa^{-1} has
    // norm <= 1 and condition <= (1 + c_k)^(1/2)), so it needs no pivoting.  Unless the right child is a leaf (which takes Us C as it is),
    // Us C is compressed through its Gram matrix when it is wider than schur_keep columns.  After the
    // right subtree, the inverse block [L^-1]_ba = -(L_bb^-1 Us)(L_aa^-T Vs)^T is formed from the
    // untruncated factors (Lf's block); L_ba itself is never truncated.
    const int ni = (int)inner.size();
    std::vector<double*> Snew(ni);
    std::vector<int*> rnew(ni);
    std::vector<int> capSb(ni), rcapv(ni), keepv(ni);
    std::vector<char> raw(ni);
    for (int i = 0; i < ni; ++i) {
      const Item& it = inner[i];
      const CholTask& T = batch[it.m];
      const Tree* t = T.Z->t;
      const int l = Tree::level(it.c);
      const int64_t sb = t->size(2 * it.c + 2);
      raw[i] = t->is_leaf(2 * it.c + 2);
      rcapv[i] = std::min(kMaxStack, T.Z->cap[l] + it.S.cap);
      if (rcapv[i] > T.Lf->cap[l]) throw std::logic_error("cholesky_inverse: Lf narrower than the stacked factors");
      keepv[i] = std::min<int>({schur_keep, (int)sb, rcapv[i]});
      capSb[i] = raw[i] ? rcapv[i] : std::max(std::min<int>({(int)sb, T.capS, kMaxStack}), keepv[i]);
      Snew[i] = scratch.get<double>((size_t)sb * capSb[i]);
      rnew[i] = scratch.get<int>(1);
    }
    // stacked factors stay allocated until the inverse blocks
    const DevArena::Mark mk = scratch.mark();
    std::vector<double*> Usv(ni), Vsv(ni);
    std::vector<int*> rsv(ni);
    {
      std::vector<StackTask> stk;
      std::vector<ThinTask> th;
      std::vector<GemmTask> gG, gC;
      std::vector<SpdCholTask> pc;
      std::vector<SymTask> sym;
      int maxrows = 1, maxsb = 1, rmax = 1;
      for (int i = 0; i < ni; ++i) {
        const Item& it = inner[i];
        const CholTask& T = batch[it.m];
        const Tree* t = T.Z->t;
        const int p = it.c, a = 2 * p + 1, b = 2 * p + 2, l = Tree::level(p);
        const int64_t sa = t->size(a), sb = t->size(b), la = t->lo[a] - t->lo[p], lb = t->lo[b] - t->lo[p];
        const int ldc = (int)t->ldf[l];
        const SF& S = it.S;
        maxrows = std::max<int>(maxrows, (int)std::max(sa, sb));
        maxsb = std::max<int>(maxsb, (int)sb);
        const int rcap = rcapv[i];
        rmax = std::max(rmax, rcap);
        double* Us = scratch.get<double>((size_t)ldc * rcap);
        double* Vs0 = scratch.get<double>((size_t)ldc * rcap);
        double* Vs = scratch.get<double>((size_t)ldc * rcap);
        // the stacked width is also the width of the untruncated inverse block [L^-1]_ba that Lf's
        // block (p, lower) receives below: the stack writes it into that block's rank slot, which
        // nothing reads before the recursion ends except through this pointer
        int* rs = T.Lf->rk(p, 1);
        Usv[i] = Us;
        Vsv[i] = Vs;
        rsv[i] = rs;
        StackTask su{};
        su.dst = Us; su.ld = ldc; su.rows = (int)sb; su.wcap = rcap; su.wout = rs; su.nsrc = 2; su.fidx = T.fidx;
        su.src[0] = {T.Z->U(p, 1), T.Z->rk(p, 1), ldc, T.Z->cap[l], 1.0};
        su.src[1] = {S.p ? S.p + lb : nullptr, S.r, S.ld, S.cap, 1.0};
        StackTask sv = su;
        sv.dst = Vs0; sv.rows = (int)sa; sv.wout = nullptr;
        sv.src[0] = {T.Z->V(p, 1), T.Z->rk(p, 1), ldc, T.Z->cap[l], 1.0};
        sv.src[1] = {S.p ? S.p + la : nullptr, S.r, S.ld, S.cap, -1.0};
        stk.push_back(su);
        stk.push_back(sv);
        th.push_back(ThinTask{view(lw[it.m]), a, Vs0, ldc, Vs, ldc, rs, rcap, 1.0, 0.0});
      }
      stack(stk, maxrows);
      keep_scratch = true;  // Vs and Us are read again by the inverse blocks
      mm_thin(th);
      keep_scratch = false;
      const DevArena::Mark mk_main = scratch.mark();
      for (int i = 0; i < ni; ++i) {
        const Item& it = inner[i];
        const CholTask& T = batch[it.m];
        const Tree* t = T.Z->t;
        const int p = it.c, a = 2 * p + 1, b = 2 * p + 2;
        const int64_t sa = t->size(a), sb = t->size(b);
        const int ldc = (int)t->ldf[Tree::level(p)], rcap = rcapv[i];
        double* G = scratch.get<double>((size_t)rcap * rcap);
        double* C = scratch.get<double>((size_t)rcap * rcap);
        int* kc = raw[i] ? rnew[i] : scratch.get<int>(1);  // a leaf child takes Us C as its factor
        GemmTask g{};  // G = Vs^T Vs
        g.A = Vsv[i]; g.opA = 1; g.lda = ldc; g.B = Vsv[i]; g.ldb = ldc; g.C = G; g.ldc = rcap;
        g.m = g.n = rcap; g.mp = g.np = rsv[i]; g.k = (int)sa; g.alpha = 1.0; g.beta = 0.0;
        gG.push_back(g);
        SpdCholTask q{};
        q.G = G; q.ldg = rcap; q.rp = rsv[i]; q.ep = T.Z->rk(p, 1); q.C = C; q.ldc = rcap; q.kout = kc; q.kcap = rcap;
        q.work = rcap > SPD_REG ? scratch.get<double>((size_t)rcap * (rcap + 1) / 2) : nullptr;
        q.fidx = T.fidx;
        pc.push_back(q);
        double* out = raw[i] ? Snew[i] : scratch.get<double>((size_t)sb * rcap);
        GemmTask c{};  // Us C
        c.A = Usv[i]; c.lda = ldc; c.B = C; c.ldb = rcap; c.C = out; c.ldc = (int)sb;
        c.m = (int)sb; c.n = rcap; c.np = kc; c.k = rcap; c.kp = rsv[i]; c.alpha = 1.0; c.beta = 0.0;
        gC.push_back(c);
        if (!raw[i]) {
          SymTask y{out, (int)sb, (int)sb, kc, rcap, Snew[i], (int)sb, rnew[i], capSb[i], thS, T.fidx};
          y.keep_below = keepv[i];
          sym.push_back(y);
        }
      }
      gemm(gG, rmax, rmax);
      launch_spd_chol(stage.upload(pc, st), (int)pc.size(), rmax, d_flag, st);
      ++launches;
      gemm(gC, maxsb, rmax);
      compress_sym(sym);
      scratch.rewind(mk_main);
    }
    // right subtrees
    std::vector<Item> right;
    for (int i = 0; i < ni; ++i) {
      const Item& it = inner[i];
      const Tree* t = batch[it.m].Z->t;
      right.push_back(Item{it.m, 2 * it.c + 2, SF{Snew[i], (int)t->size(2 * it.c + 2), rnew[i], capSb[i]}});
    }
    dfs(right);
    // inverse blocks from the untruncated factors: U = -L_bb^{-1} Us, V = L_aa^{-T} Vs, rank = width
    const DevArena::Mark mk2 = scratch.mark();
    std::vector<ThinTask> th;
    for (int i = 0; i < ni; ++i) {
      const Item& it = inner[i];
      const CholTask& T = batch[it.m];
      const int p = it.c, a = 2 * p + 1, b = 2 * p + 2, l = Tree::level(p);
      const int ldc = (int)T.Z->t->ldf[l];
      th.push_back(ThinTask{view(lw[it.m]), b, Usv[i], ldc, T.Lf->U(p, 1), ldc, rsv[i], rcapv[i], -1.0, 0.0});
      th.push_back(ThinTask{view(lw[it.m], true), a, Vsv[i], ldc, T.Lf->V(p, 1), ldc, rsv[i], rcapv[i], 1.0, 0.0});
    }
    mm_thin(th);
    // the factor's own block L_ba = Us Vs^T, where the caller keeps L
    std::vector<StackTask> lc;
    int lrows = 1;
    for (int i = 0; i < ni; ++i) {
      const Item& it = inner[i];
      const CholTask& T = batch[it.m];
      if (!T.L) continue;
      const Tree* t = T.Z->t;
      const int p = it.c, l = Tree::level(p);
      const int ldc = (int)t->ldf[l];
      const int64_t sa = t->size(2 * p + 1), sb = t->size(2 * p + 2);
      StackTask u{};
      u.dst = T.L->U(p, 1); u.ld = ldc; u.rows = (int)sb; u.wcap = T.L->cap[l]; u.wout = T.L->rk(p, 1); u.nsrc = 1;
      u.fidx = T.fidx;
      u.src[0] = {Usv[i], rsv[i], ldc, rcapv[i], 1.0};
      StackTask v = u;
      v.dst = T.L->V(p, 1); v.rows = (int)sa; v.wout = nullptr;
      v.src[0] = {Vsv[i], rsv[i], ldc, rcapv[i], 1.0};
      lc.push_back(u);
      lc.push_back(v);
      lrows = std::max<int>(lrows, (int)std::max(sa, sb));
    }
    stack(lc, lrows);
    scratch.rewind(mk2);
    scratch.rewind(mk);
  };
  std::vector<Item> roots;
  for (int m = 0; m < (int)batch.size(); ++m) roots.push_back(Item{m, 0, SF{nullptr, 1, d_zero, 0}});
  dfs(roots);
  // truncated recompression of every inverse block, all levels and members at once
  std::vector<RecTask> rec;
  for (const CholTask& T : batch) {
    const Tree* t = T.Z->t;
    for (int p = 0; p < t->ninternal; ++p) {
      const int l = Tree::level(p), ld = (int)t->ldf[l];
      RecTask r{};
      r.Us = T.Lf->U(p, 1); r.ldus = ld; r.m = (int)t->size(2 * p + 2);
      r.Vs = T.Lf->V(p, 1); r.ldvs = ld; r.n = (int)t->size(2 * p + 1);
      r.r = T.Lf->rk(p, 1); r.rcap = T.Lf->cap[l];
      r.U = T.Linv->U(p, 1); r.V = T.Linv->V(p, 1); r.ldu = r.ldv = ld; r.rank = T.Linv->rk(p, 1);
      r.kcap = T.Linv->cap[l]; r.thresh = tol; r.fidx = T.fidx;
      rec.push_back(r);
    }
  }
  recompress(rec);
}

void Engine::trsm_thin(const HMat& L, bool trans, double* B, int ldb, double* Z, int ldz, const int* w, int wcap,
                       int p) {
  const Tree& t = *L.t;
  const int64_t lo = t.lo[p];
  if (t.is_leaf(p)) {  // Z_i = L_i^{-1} B_i (or L_i^{-T} B_i)
    const int m = (int)t.size(p);
    GemmTask g{};
    g.A = L.leaf(t.leaf_index(p)); g.lda = L.ldl; g.opA = trans ? 1 : 0;
    g.B = B + lo; g.ldb = ldb; g.C = Z + lo; g.ldc = ldz;
    g.m = m; g.k = m; g.n = wcap; g.np = w; g.alpha = 1.0; g.beta = 0.0;
    gemm({g}, m, wcap);
    return;
  }
  const int a = 2 * p + 1, b = 2 * p + 2, l = Tree::level(p), ld = (int)t.ldf[l], cap = L.cap[l];
  const int64_t la = t.lo[a], lb = t.lo[b];
  const int sa = (int)t.size(a), sb = (int)t.size(b);
  const DevArena::Mark mk = scratch.mark();
  double* tmp = scratch.get<double>((size_t)std::max(cap, 1) * wcap);
  // L = [L_aa 0; L_ba L_bb], L_ba = U V^T (block (p, lower)).  Forward: Z_a, then
  // B_b -= U (V^T Z_a), then Z_b.  Transposed (L^T upper): Z_b, then B_a -= V (U^T Z_b), then Z_a.
  const int first = trans ? b : a, second = trans ? a : b;
  trsm_thin(L, trans, B, ldb, Z, ldz, w, wcap, first);
  const double* Pz = Z + (trans ? lb : la);   // solved part
  double* Bu = B + (trans ? la : lb);          // part to update
  const double* Left = trans ? L.V(p, 1) : L.U(p, 1);    // rows of the updated part
  const double* Right = trans ? L.U(p, 1) : L.V(p, 1);   // rows of the solved part
  GemmTask g1{};  // tmp = Right^T Z_solved  (cap x w)
  g1.A = Right; g1.opA = 1; g1.lda = ld; g1.B = Pz; g1.ldb = ldz; g1.C = tmp; g1.ldc = std::max(cap, 1);
  g1.m = cap; g1.mp = L.rk(p, 1); g1.n = wcap; g1.np = w; g1.k = trans ? sb : sa; g1.alpha = 1.0; g1.beta = 0.0;
  gemm({g1}, cap, wcap);
  GemmTask g2{};  // B_upd -= Left tmp
  g2.A = Left; g2.lda = ld; g2.B = tmp; g2.ldb = std::max(cap, 1); g2.C = Bu; g2.ldc = ldb;
  g2.m = trans ? sa : sb; g2.n = wcap; g2.np = w; g2.k = cap; g2.kp = L.rk(p, 1); g2.alpha = -1.0; g2.beta = 1.0;
  gemm({g2}, g2.m, wcap);
  scratch.rewind(mk);
  trsm_thin(L, trans, B, ldb, Z, ldz, w, wcap, second);
}

std::vector<int> Engine::chol_work_caps(const Tree& t, const std::vector<int>& capZ, int capS) const {
  std::vector<int> c(t.L, 1);
  for (int l = 0; l < t.L && l < (int)capZ.size(); ++l)
    c[l] = std::min(kMaxStack, capZ[l] + std::max(capS, schur_keep));
  return c;
}

// ---------------------------------------------------------------------------------------------
void Engine::sym_affine(const std::vector<AffTask>& batch) {
  std::vector<StackTask> stk, cp;
  std::vector<RecTask> rec;
  std::vector<LeafAxpy> ax;
  int maxrows = 1, maxleaf = 1;
  for (const AffTask& A : batch) {
    const Tree* t = A.X->t;
    HMat& P = *A.P;
    const double sx = A.sx;
    zero_ranks(P);
    const HView Xv = view(*A.X);
    for (int p = 0; p < t->ninternal; ++p) {
      const int l = Tree::level(p), ldc = (int)t->ldf[l];
      const int64_t sa = t->size(2 * p + 1), sb = t->size(2 * p + 2);
      maxrows = std::max<int>(maxrows, (int)std::max(sa, sb));
      const HView::Blk u = Xv.upper(p), lo = Xv.lower(p);
      const int rcap = std::min(kMaxStack, u.cap + lo.cap);
      double* Us = scratch.get<double>((size_t)ldc * rcap);
      double* Vs = scratch.get<double>((size_t)ldc * rcap);
      int* rs = scratch.get<int>(1);
      StackTask su{};
      su.dst = Us; su.ld = ldc; su.rows = (int)sa; su.wcap = rcap; su.wout = rs; su.nsrc = 2; su.fidx = A.fidx;
      su.src[0] = {u.U, u.r, u.ld, u.cap, 0.5 * sx};
      su.src[1] = {lo.V, lo.r, lo.ld, lo.cap, 0.5 * sx};
      StackTask sv = su;
      sv.dst = Vs; sv.rows = (int)sb; sv.wout = nullptr;
      sv.src[0] = {u.V, u.r, u.ld, u.cap, 1.0};
      sv.src[1] = {lo.U, lo.r, lo.ld, lo.cap, 1.0};
      stk.push_back(su);
      stk.push_back(sv);
      RecTask r{};
      r.Us = Us; r.ldus = ldc; r.m = (int)sa; r.Vs = Vs; r.ldvs = ldc; r.n = (int)sb; r.r = rs; r.rcap = rcap;
      r.U = P.U(p, 0); r.V = P.V(p, 0); r.ldu = r.ldv = ldc; r.rank = P.rk(p, 0); r.kcap = P.cap[l]; r.thresh = tol;
      r.fidx = A.fidx;
      rec.push_back(r);
      // lower block = transpose of the upper one (issued after the recompression)
      StackTask a{};
      a.dst = P.U(p, 1); a.ld = ldc; a.rows = (int)sb; a.wcap = P.cap[l]; a.wout = P.rk(p, 1); a.nsrc = 1; a.fidx = A.fidx;
      a.src[0] = {P.V(p, 0), P.rk(p, 0), ldc, P.cap[l], 1.0};
      StackTask b = a;
      b.dst = P.V(p, 1); b.rows = (int)sa; b.wout = nullptr;
      b.src[0] = {P.U(p, 0), P.rk(p, 0), ldc, P.cap[l], 1.0};
      cp.push_back(a);
      cp.push_back(b);
    }
    for (int q = t->ninternal; q < t->nnodes; ++q) {
      const int li = t->leaf_index(q);
      LeafAxpy x{};
      x.out = P.leaf(li); x.ldo = P.ldl; x.X = A.X->leaf(li); x.ldx = A.X->ldl; x.Y = A.X->leaf(li); x.ldy = A.X->ldl;
      x.transY = 1; x.m = (int)t->size(q); x.alpha = 0.5 * sx; x.beta = 0.5 * sx; x.gamma = A.sid;
      ax.push_back(x);
    }
    maxleaf = std::max(maxleaf, (int)t->maxleaf);
  }
  stack(stk, maxrows);
  recompress(rec);
  stack(cp, maxrows);
  if (!ax.empty()) {
    launch_leaf_axpy(stage.upload(ax, st), (int)ax.size(), maxleaf, st);
    ++launches;
  }
}

void Engine::sum(const std::vector<SumTask>& batch) {
  if (batch.empty()) return;
  std::vector<StackTask> stk;
  std::vector<RecTask> rec;
  int maxrows = 1, ldlmax = 1, nmax = 0;
  for (const SumTask& T : batch) {
    const int nt = (int)T.terms.size();
    if (nt < 1 || nt > kStackSrc) throw std::invalid_argument("Engine::sum: 1 to kStackSrc terms");
    const Tree* t = T.C->t;
    for (const auto& w : T.terms)
      if (w.second->t != t || w.second->lower_only) throw std::invalid_argument("Engine::sum: terms of another tree");
    nmax = std::max(nmax, nt);
    ldlmax = std::max(ldlmax, (int)t->maxleaf);
    for (int p = 0; p < t->ninternal; ++p) {
      const int l = Tree::level(p), ldc = (int)t->ldf[l];
      const int64_t sa = t->size(2 * p + 1), sb = t->size(2 * p + 2);
      maxrows = std::max<int>(maxrows, (int)std::max(sa, sb));
      int rcap = 0;
      for (const auto& w : T.terms) rcap += w.second->cap[l];
      rcap = std::max(1, std::min(kMaxStack, rcap));  // wider: flagged by k_stack
      for (int s = 0; s < 2; ++s) {
        const int64_t mr = s == 0 ? sa : sb, mc = s == 0 ? sb : sa;
        double* Us = scratch.get<double>((size_t)ldc * rcap);
        double* Vs = scratch.get<double>((size_t)ldc * rcap);
        int* rs = scratch.get<int>(1);
        StackTask su{};
        su.dst = Us; su.ld = ldc; su.rows = (int)mr; su.wcap = rcap; su.wout = rs; su.nsrc = nt; su.fidx = T.fidx;
        StackTask sv = su;
        sv.dst = Vs; sv.rows = (int)mc; sv.wout = nullptr;
        for (int i = 0; i < nt; ++i) {
          const HMat& H = *T.terms[i].second;
          su.src[i] = {H.U(p, s), H.rk(p, s), ldc, H.cap[l], T.terms[i].first};
          sv.src[i] = {H.V(p, s), H.rk(p, s), ldc, H.cap[l], 1.0};
        }
        stk.push_back(su);
        stk.push_back(sv);
        RecTask r{};
        r.Us = Us; r.ldus = ldc; r.m = (int)mr; r.Vs = Vs; r.ldvs = ldc; r.n = (int)mc; r.r = rs; r.rcap = rcap;
        r.U = T.C->U(p, s); r.V = T.C->V(p, s); r.ldu = r.ldv = ldc; r.rank = T.C->rk(p, s); r.kcap = T.C->cap[l];
        r.thresh = tol; r.fidx = T.fidx;
        rec.push_back(r);
      }
    }
  }
  stack(stk, maxrows);
  recompress(rec);
  // leaves: out = w_0 T_0 + w_1 T_1, then out += w_i T_i, one launch per term for all leaves
  for (int i = 0; i == 0 || i < nmax; i = i == 0 ? 2 : i + 1) {
    std::vector<LeafAxpy> ax;
    for (const SumTask& T : batch) {
      const int nt = (int)T.terms.size();
      if (i > 0 && i >= nt) continue;
      const Tree* t = T.C->t;
      for (int q = t->ninternal; q < t->nnodes; ++q) {
        const int li = t->leaf_index(q);
        LeafAxpy x{};
        x.out = T.C->leaf(li); x.ldo = T.C->ldl; x.m = (int)t->size(q);
        if (i == 0) {
          x.X = T.terms[0].second->leaf(li); x.ldx = T.terms[0].second->ldl; x.alpha = T.terms[0].first;
          if (nt > 1) {
            x.Y = T.terms[1].second->leaf(li); x.ldy = T.terms[1].second->ldl; x.beta = T.terms[1].first;
          }
        } else {
          x.X = x.out; x.ldx = x.ldo; x.alpha = 1.0;
          x.Y = T.terms[i].second->leaf(li); x.ldy = T.terms[i].second->ldl; x.beta = T.terms[i].first;
        }
        ax.push_back(x);
      }
    }
    if (!ax.empty()) {
      launch_leaf_axpy(stage.upload(ax, st), (int)ax.size(), ldlmax, st);
      ++launches;
    }
  }
}

void Engine::copy_hmat(const HMat& src, HMat& dst) {
  const Tree* t = src.t;
  HQ_CHECK(hipMemcpyAsync(dst.leaves, src.leaves, sizeof(double) * (size_t)t->nleaves * src.ldl * src.ldl,
                          hipMemcpyDeviceToDevice, st));
  for (int l = 0; l < t->L; ++l) {
    if (src.cap[l] != dst.cap[l]) throw std::runtime_error("copy_hmat: capacity mismatch");
    const size_t per = (size_t)(2 << l) * t->ldf[l] * src.cap[l] * sizeof(double);
    HQ_CHECK(hipMemcpyAsync(dst.Ubase[l], src.Ubase[l], per, hipMemcpyDeviceToDevice, st));
    HQ_CHECK(hipMemcpyAsync(dst.Vbase[l], src.Vbase[l], per, hipMemcpyDeviceToDevice, st));
  }
  launch_copy_int(dst.rank, src.rank, 2 * t->ninternal, st);
}

}  // namespace hq

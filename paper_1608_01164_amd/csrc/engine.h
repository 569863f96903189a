// HODLR engine: cluster tree, device storage of HODLR matrices, and the formatted operations of
// the QDWH iteration (Sec. 3.1.1 of the paper: products with recompression, Cholesky, triangular
// solves), issued as batched kernel launches on the caller's stream and three side streams.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"

namespace hq {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
#define HQ_CHECK(x)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) throw ::hq::HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Binary cluster tree in heap order: node 0 is [0, n); node p splits [lo, hi) at
// lo + ceil((hi - lo)/2) into children 2p+1, 2p+2.  All leaves sit at level L, the smallest
// level whose blocks have at most `leaf` rows (Sec. 3.1.1: stop once n/2^l <= n_min).
struct Tree {
  int64_t n = 0;
  int leaf = 0, L = 0;
  int nnodes = 0, ninternal = 0, nleaves = 0;
  int64_t maxleaf = 0;
  std::vector<int64_t> lo, hi;
  std::vector<int64_t> ldf;  // per level l < L: largest child size (leading dim of factors)
  void build(int64_t n_, int leaf_);
  int64_t size(int p) const { return hi[p] - lo[p]; }
  int64_t mid(int p) const { return lo[p] + (hi[p] - lo[p] + 1) / 2; }
  static int level(int p) {
    int l = 0;
    while ((2 << l) - 1 <= p) ++l;
    return l;
  }
  bool is_leaf(int p) const { return p >= ninternal; }
  int leaf_index(int p) const { return p - ninternal; }
};

// Device bump allocator over large chunks (256-byte aligned).
class DevArena {
 public:
  DevArena() = default;
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  ~DevArena();
  void* alloc(size_t bytes);
  template <class T>
  T* get(size_t count) { return static_cast<T*>(alloc(sizeof(T) * (count ? count : 1))); }
  void reset();  // keeps chunks, rewinds
  // Serve every request from one caller-owned device buffer of `cap` bytes (256-byte aligned), never
  // from the runtime: a request beyond it throws NoAlloc.  The buffer is not released.
  void attach_fixed(void* p, size_t cap);
  void swap(DevArena& o) {
    chunks_.swap(o.chunks_);
    std::swap(cur_, o.cur_);
    std::swap(inuse_, o.inuse_);
    std::swap(high_, o.high_);
    std::swap(chunk_bytes, o.chunk_bytes);
    std::swap(fixed_, o.fixed_);
  }
  struct Mark { size_t cur, used, inuse; };
  Mark mark() const { return Mark{cur_, cur_ < chunks_.size() ? chunks_[cur_].used : 0, inuse_}; }
  void rewind(const Mark& m);  // memory handed out after m may be reused (stream order keeps it safe)
  size_t high_water() const { return high_; }
  size_t chunk_bytes = size_t(256) << 20;

 private:
  struct Chunk { char* p; size_t cap, used; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, inuse_ = 0, high_ = 0;
  bool fixed_ = false;  // chunks_ is one external buffer
};

// A request that an allocation-free call cannot serve from its fixed buffers.
struct NoAlloc : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Device memory free for this library's use: the runtime's free memory plus the chunks kept for
// reuse by earlier calls.
size_t free_device_bytes();

// Pinned host block taken from the chunk cache and handed back to it (once the device has drained)
// when the object goes; host images of matrices are built in place in it and copied to the device
// without a staging copy.
class PinnedHost {
 public:
  explicit PinnedHost(size_t bytes);
  PinnedHost(const PinnedHost&) = delete;
  PinnedHost& operator=(const PinnedHost&) = delete;
  ~PinnedHost();
  template <class T>
  T* as() const { return reinterpret_cast<T*>(p_); }
 private:
  char* p_ = nullptr;
  size_t cap_ = 0;
};

// Task descriptors in pinned host memory that the kernels read directly.
class DescStage {
 public:
  DescStage() = default;
  DescStage(const DescStage&) = delete;
  DescStage& operator=(const DescStage&) = delete;
  ~DescStage();
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s) { return static_cast<T*>(up(v.data(), sizeof(T) * v.size(), s)); }
  void reset();  // only after the stream has drained
  // Make sure one chunk of at least `bytes` exists (allocating if needed), so that later uploads of
  // up to that size in total, after a reset(), take no new pinned memory.
  void reserve(size_t bytes);
  size_t capacity() const;
  bool no_grow = false;  // set: an upload that needs a new chunk throws NoAlloc instead
 private:
  void* up(const void* src, size_t bytes, hipStream_t s);
  struct Chunk { char* h; size_t cap, used; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
};

// A HODLR matrix on the device.  Block s of internal node p: s = 0 upper (rows = left child a,
// cols = right child b), s = 1 lower (rows b, cols a); stored as U (rows x cap) V (cols x cap)
// with leading dimension ldf[level] and a device rank.
struct HMat {
  const Tree* t = nullptr;
  std::vector<int> cap;           // per level
  int ldl = 0;
  double* leaves = nullptr;
  std::vector<double*> Ubase, Vbase;
  int* rank = nullptr;            // 2 * ninternal
  bool lower_only = false;        // symmetric storage: upper blocks implied by transposition
  double* leaf(int li) const { return leaves + (size_t)li * ldl * ldl; }
  double* U(int p, int s) const {
    const int l = Tree::level(p), i = p - ((1 << l) - 1);
    return Ubase[l] + (size_t)(2 * i + s) * t->ldf[l] * cap[l];
  }
  double* V(int p, int s) const {
    const int l = Tree::level(p), i = p - ((1 << l) - 1);
    return Vbase[l] + (size_t)(2 * i + s) * t->ldf[l] * cap[l];
  }
  int* rk(int p, int s) const { return rank + 2 * p + s; }
  int ld(int p) const { return (int)t->ldf[Tree::level(p)]; }
  int capof(int p) const { return cap[Tree::level(p)]; }
  size_t bytes() const;
};

// op(H) as seen by an operation: trans swaps the roles of the two blocks and of U and V.
struct HView {
  const HMat* h = nullptr;
  bool trans = false;
  const int* zero = nullptr;  // device int holding 0 (used for blocks known to vanish)
  struct Blk { const double* U; const double* V; const int* r; int ld, cap; };
  Blk upper(int p) const;  // rows a, cols b of op(H)
  Blk lower(int p) const;  // rows b, cols a of op(H)
  HView T() const { HView v = *this; v.trans = !trans; return v; }
};

// Row tiling of the R-only TSQR of an m-row stack with rcap columns of capacity.
struct QrPlan { int h0, hs, ntiles; };
QrPlan plan_qr(int m, int rcap);

struct Thin {            // dense n_sub x w block (column-major) with a device width
  double* p; int ld; const int* w; int wcap;
};

class Engine {
 public:
  static constexpr int kFlagSlots = 1024;  // one status word per matrix of a batch
  explicit Engine(hipStream_t s);
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine();
  hipStream_t st;
  // Further streams (default priority) for work off the critical path: the recompression of L_ba in
  // the H-Cholesky, the C blocks of each level of a product.  Created on first use; work issued there
  // is always joined back into st before its memory is released.
  static constexpr int kSides = 3;
  hipStream_t side_stream(int i);
  // The H-Cholesky's lazy Schur factor is compressed (through its Gram matrix) only when it has more
  // live columns than this; narrower factors are carried as they are.
  int schur_keep = 96;
  bool keep_scratch = false;  // set while issuing side-stream work: helpers then keep their workspace
  DevArena persist, scratch;
  DescStage stage;
  // d_flag[i], status of batch member i: bit 0 rank overflow, bit 1 not positive definite, bit 2 stack
  // overflow, bit 3 non-finite singular values, bit 4 non-finite stacked factors, bit 5 non-finite R
  int* d_flag = nullptr;
  int* d_zero = nullptr;
  double tol = 1e-10;
  int64_t launches = 0;
  // Compute precision of the GEMM, TSQR and core-SVD kernels issued from now on (factors stay
  // FP64 in memory; FP32 kernels round operands on load and truncate at max(tol, 8 u32 sigma_1)).
  bool fp32 = false;

  HMat alloc_hmat(const Tree* t, const std::vector<int>& cap, bool lower_only = false) {
    return alloc_hmat_in(persist, t, cap, lower_only);
  }
  HMat alloc_hmat_in(DevArena& ar, const Tree* t, const std::vector<int>& cap, bool lower_only = false);
  HView view(const HMat& h, bool trans = false) const { HView v; v.h = &h; v.trans = trans; v.zero = d_zero; return v; }
  void zero_ranks(HMat& h);

  // Y[rows of root] = alpha * op(H)|root * X + beta * Y for a list of subtree tasks.
  struct ThinTask {
    HView H; int root; const double* X; int ldx; double* Y; int ldy; const int* w; int wcap; double alpha, beta;
  };
  void mm_thin(const std::vector<ThinTask>& tasks);

  // Stream capture of everything issued between capture_begin and capture_end_launch (the library
  // stream and the side streams it forks and joins) into one HIP graph, which is instantiated and
  // launched on the library stream.  The executable graph lives until release(), which the caller
  // issues after the stream has drained.
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    int64_t nodes = 0;
    double build_seconds = 0.0;
    void release();
    Graph() = default;
    Graph(const Graph&) = delete;
    Graph& operator=(const Graph&) = delete;
    Graph(Graph&& o) noexcept { *this = std::move(o); }
    Graph& operator=(Graph&& o) noexcept {
      if (this != &o) {
        release();
        g = o.g; x = o.x; nodes = o.nodes; build_seconds = o.build_seconds;
        o.g = nullptr;
        o.x = nullptr;
      }
      return *this;
    }
    ~Graph() { release(); }
  };
  void capture_begin();
  Graph capture_end_launch();
  bool capturing = false;
  hipStream_t cap_stream = nullptr, caller_st = nullptr;
  std::chrono::steady_clock::time_point cap_t0;
  // Device workspace mm_thin takes from `scratch` for these tasks (block-sized V^T X buffers, then
  // the largest split-K workspace of its launches), in the arena's 256-byte granules.
  static size_t thin_scratch_bytes(const std::vector<ThinTask>& tasks);

  // Truncated recompression of stacked factors Us (m x r) Vs (n x r) into (U, V, rank):
  // U' = Us Rv^T J_k (scaled by sigma), V' = Vs Ru^T (B J)_k / sigma^2 (orthonormal columns).
  struct RecTask {
    const double* Us; int ldus; int m;
    const double* Vs; int ldvs; int n;
    const int* r; int rcap;
    double* U; double* V; int ldu, ldv; int* rank; int kcap;
    double thresh;
    int fidx;
    const double* Rv = nullptr;  // R factor of Vs (rcap x rcap, ld rcap) when already computed
  };
  void recompress(const std::vector<RecTask>& tasks);
  // R factor (rcap x rcap, ld rcap) of each stack M (rows x live r), by the TSQR of recompress.
  struct QrJob { const double* M; int ldm; int rows; const int* r; int rcap; double* R; int fidx; };
  void qr_r(const std::vector<QrJob>& jobs);
  size_t rec_budget = size_t(3) << 30;  // device workspace of one group of recompressions
  // Symmetric factor compression: S (m x r) -> S J_k with S S^T ~ S' S'^T, drop sigma(S) <= thresh.
  struct SymTask {
    const double* S; int lds; int m; const int* r; int rcap; double* out; int ldo; int* rank; int kcap; double thresh;
    int fidx;
    int keep_below = 0;  // a factor of at most this many live columns is kept as it is (out = S)
  };
  void compress_sym(const std::vector<SymTask>& tasks);
  // `core_after`: the stream waits for it between the TSQR and the core of the group (a task's Rv
  // may be produced on another stream).
  void recompress_group(const std::vector<RecTask>& tasks, hipEvent_t core_after = nullptr);
  void compress_sym_group(const std::vector<SymTask>& tasks);

  // C = alpha op(A) op(B) + delta op(D)  (D absent, a HODLR, or the identity), for a batch of
  // independent matrices: every launch covers all members.
  struct ProdTask {
    HView A, B, D;      // D.h == nullptr: no D term
    bool d_identity = false;
    double alpha = 1.0, delta = 0.0;
    HMat* C = nullptr;
    int fidx = 0;
  };
  void product(const std::vector<ProdTask>& v);
  void product(HView A, HView B, const HView* D, bool d_identity, double alpha, double delta, HMat& C);
  // Cholesky Z = L L^T of symmetric HODLR matrices (lower blocks + leaves); L^{-1} in Linv.  The
  // members' recursions advance in lockstep, one launch per step for all of them.
  // Z = L L^T and Linv = L^{-1} (capacities of the truncated inverse).  Lf: workspace of the same
  // tree whose leaves receive the leaf factors and whose off-diagonal blocks receive the untruncated
  // inverse blocks; its capacities must be chol_work_caps(Z's capacities, capS).  capS: capacity of
  // the compressed Schur factor.
  // L (optional): receives the factor's off-diagonal blocks L_ba = Us Vs^T, untruncated (capacities
  // of Lf); its leaves are Linv's (the inverses of the diagonal blocks), which is what substitution
  // with L needs.
  struct CholTask { const HMat* Z; HMat* Linv; HMat* Lf; int capS; int fidx; HMat* L = nullptr; };
  std::vector<int> chol_work_caps(const Tree& t, const std::vector<int>& capZ, int capS) const;
  void cholesky_inverse(const std::vector<CholTask>& v);
  void leaf_chol_inv(const std::vector<LeafTask>& blocks);
  void cholesky_inverse(const HMat& Z, HMat& Linv, HMat& Lf, int capS) { cholesky_inverse({CholTask{&Z, &Linv, &Lf, capS, 0}}); }
  // Triangular solve with a thin dense right-hand side by substitution over the tree (Table
  // complexity_HODLR: HODLR times triangular = given): L Z = B (trans false) or L^T Z = B (trans
  // true), L lower triangular with the inverses of its diagonal blocks as leaves (CholTask::L).  B
  // (n x w, leading dimension ldb) is overwritten by the updates, Z receives the solution.  Depth
  // first: one GEMM per leaf and two per off-diagonal block, in dependency order.
  void trsm_thin(const HMat& L, bool trans, double* B, int ldb, double* Z, int ldz, const int* w, int wcap, int p = 0);
  // out = sid * I + sx * (X + X^T) / 2 as a full HODLR (sign: sx = 1, sid = 0; projector: -1/2, 1/2)
  // C = sum_i w_i T_i (general HODLR matrices of one tree, at most kStackSrc terms): each block's
  // factors stacked with the weights on the U side and recompressed at tol; leaves summed.
  struct SumTask { std::vector<std::pair<double, const HMat*>> terms; HMat* C; int fidx; };
  void sum(const std::vector<SumTask>& v);
  struct AffTask { const HMat* X; HMat* P; double sx, sid; int fidx; };
  void sym_affine(const std::vector<AffTask>& v);
  void sym_affine(const HMat& X, HMat& P, double sx, double sid) { sym_affine({AffTask{&X, &P, sx, sid, 0}}); }
  void copy_hmat(const HMat& src, HMat& dst);

  int read_flag() { return read_flags(1)[0]; }
  std::vector<int> read_flags(int count);
  void clear_flag() { clear_flags(1); }
  void clear_flags(int count);
  std::vector<int> read_ranks(const HMat& h);

  // helpers
  hipEvent_t take_event();
  void give_event(hipEvent_t e) { ev_free.push_back(e); }
  void gemm(const std::vector<GemmTask>& v, int max_m, int max_n);
  void stack(const std::vector<StackTask>& v, int max_rows);

 private:
  std::vector<hipEvent_t> ev_all, ev_free;
  hipStream_t sides_[kSides] = {};
  int next_side = 0;

 public:
  // Workspace of the product's C blocks issued on side stream k: reset when stream k is next used
  // for them (stream order makes the reuse safe), so at most kSides levels hold buffers at a time.
  DevArena side_arena[kSides];
  size_t side_high_water() const {
    size_t h = 0;
    for (const DevArena& a : side_arena) h += a.high_water();
    return h;
  }
};

}  // namespace hq

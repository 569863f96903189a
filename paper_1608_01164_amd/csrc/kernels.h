// Device kernels of the HODLR-QDWH path (gfx950).  Host-side launch wrappers.
//
// Every batched kernel takes an array of task descriptors in device memory.  Sizes that are
// only known on the device (off-diagonal ranks, stacked widths) are read through `const int*`
// fields; the matching static field is then an upper bound used to size the grid, and tiles
// beyond the live size exit at once.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hq {

// Kernel classes for the built-in timers (HIP events around each launch, on the launch stream)
// and the device-side counters of algorithmic work (flops and operand bytes per launch).
enum KClass { K_GEMM = 0, K_QR, K_SVD, K_POTRF, K_TRTRI, K_STACK, K_LEAF, K_OTHER, K_NCLASS };
struct ProfStat {
  long long launches;
  double ms, flops, bytes;
};
void prof_enable(bool on);
void prof_select(unsigned mask);  // classes whose launches get timers (bit c for class c; default all)
bool prof_enabled();
void prof_read(ProfStat out[K_NCLASS], bool reset);
void prof_mfma(double out[2], bool reset);  // flops issued to the matrix cores, FP64 and FP32
void prof_svd_stats(unsigned long long out[8]);  // core-SVD phase cycles and sizes (test/bench aid)
int prof_begin(int cls, hipStream_t s);    // a record slot, or -1 when profiling is off for cls
void prof_end(int slot, hipStream_t s);

// C = alpha * op(A) * op(B) + beta * C, column-major, op = N (0) or T (1).
struct GemmTask {
  const double* A;
  const double* B;
  double* C;
  const int* mp;  // if non-null, m = *mp (else m)
  const int* np;
  const int* kp;
  int m, n, k;    // static sizes (upper bounds when the pointer is set)
  int lda, ldb, ldc;
  int opA, opB;
  double alpha, beta;
  double* W;      // split-K: partial tiles (splits per output tile), summed in order by a second kernel
  int splits;     // K ranges when W is set
  const double* Cin;  // if non-null, beta scales Cin (leading dimension ldcin) instead of C: C = alpha AB + beta Cin
  int ldcin;
};
// K ranges of a product whose k is a true dimension (no device count): a function of k alone, so
// that a task's result never depends on what else shares its launch or on any capacity.
// Tile shapes and thresholds picked by the project's autotuner: read once from the table next to the
// library (tuning.txt, "key value" lines) or the file named by HQ_TUNING; these are the defaults.
struct Tuning {
  int qr_tile_rows = 1024;  // rows of a TSQR row tile (stage 0)
  int split_min_k = 512;    // split-K GEMM only for k >= this
  int split_chunk = 256;    // rows of K per split
  int split_max = 32;       // most splits
  int schur_keep = 96;      // H-Cholesky: Schur factors up to this width are carried uncompressed
  int gemm_small_tiles = 64;  // GEMM launches of at most this many 64 x 64 tiles (no split-K) use 32 x 32 tiles
  bool valid() const {
    return qr_tile_rows >= 32 && qr_tile_rows <= 8192 && split_min_k >= 64 && split_chunk >= 32 && split_max >= 1 &&
           split_max <= 128 && schur_keep >= 0 && schur_keep <= 1024 && gemm_small_tiles >= 0 &&
           gemm_small_tiles <= (1 << 20);
  }
};
Tuning& tuning();
inline int gemm_splits(int k) {
  const Tuning& t = tuning();
  if (k < t.split_min_k) return 1;
  const int s = k / t.split_chunk;
  return s < 1 ? 1 : (s < t.split_max ? s : t.split_max);
}

// dst[:, off_s : off_s + w_s] = scale_s * src_s[:, 0 : w_s] for s = 0..nsrc-1, off_s = sum of previous widths.
// Widest stack of factor columns the recompression kernels take (TSQR and core SVD limits).
constexpr int kMaxStack = 1024;

struct StackSrc {
  const double* p;
  const int* wp;  // dynamic width (or null -> w)
  int ld, w;
  double scale;
};
constexpr int kStackSrc = 10;  // most sources of one stack (a sum of up to nine terms and a D block)
struct StackTask {
  double* dst;
  int* wout;      // receives the total width (may be null)
  int ld, rows, nsrc, wcap;  // wcap: capacity of dst in columns (overflow -> flag[fidx])
  int fidx;
  StackSrc src[kStackSrc];
};

// R-only Householder QR of a tall matrix, tree-reduced (TSQR).  Stage 0 copies a row tile of
// the source into a workspace slot and triangularises it; stage s >= 1 stacks the triangle of
// slot i + 2^(s-1) under that of slot i and triangularises again.  After the last stage slot 0
// holds R (min(rows, r) x r, upper trapezoidal), copied to R (ldr) with zero padding to r x r.
// In FP64 a single-tile stack with rows <= r is its own factor (M = I M) and is passed on
// unfactored, so R is then the stack itself; what the recompression needs holds either way: M = Q R with Q
// orthonormal columns, i.e. R^T R = M^T M.
struct QrTask {
  const double* M;   // source (rows x r), ld = ldm
  const int* rp;     // live column count r
  double* work;      // ntiles slots of (hs x rcap)
  double* R;         // output r x r
  int ldm, rows, rcap, hs, h0, ntiles, ldr;
  int fidx;          // status word of the owning matrix (non-finite input 16, non-finite R 32)
};

// Truncated SVD of the small core B (r x r): Householder QR with column pivoting of B, stopped
// once the trailing block's Frobenius norm is below qr_thresh (B Pi ~ Q_t R_t), then one-sided
// Jacobi on R_t^T (r x t) with accumulated rotations J (t x t), sorted, truncated at
// sigma > thresh and capped at kcap (overflow -> flag bit 0).  With B ~ U S V^T:
//   Jk = V_k (r x k'),   Wk = U_k S_k^{-1} (r x k').
struct SvdTask {
  double* B;         // r x r, destroyed
  double* C;         // r x r workspace
  double* Jw;        // r x r workspace (rotations when t exceeds the LDS copy)
  double* aux;       // 2r workspace
  double* Wk;        // r x kcap output (null: the left singular vectors are not formed)
  double* Jk;        // r x kcap output
  double* sig;       // r sorted singular values (may be null)
  const int* rp;
  int* kout;         // receives k'
  int ld, kcap;
  double thresh, qr_thresh;
  int fidx;          // status word of the owning matrix (rank overflow sets bit 0)
  float fp32_floor;  // FP32 variant: truncate below max(thresh, fp32_floor * sigma_1)
  // Rows and columns of B at or beyond rlim are zero (the core of a block with fewer rows than
  // stacked columns): the decomposition runs on the leading min(r, rlim) square, and rows from
  // there to r of Wk and Jk come out zero.
  int rlim = 1 << 30;
  // A core of live order r <= keep_below is kept as it is: Jk = the first r columns of the identity,
  // k' = r (Wk and sig are not written).  0: always decompose.
  int keep_below = 0;
};

// Cholesky M = C C^T (C lower, r x r) of a small symmetric positive definite M = G + E, where G is a
// Gram matrix (both triangles stored) and E = 1 on the diagonal from index *ep on, 0 before.  The
// H-Cholesky's M is positive definite by construction (see the engine), so no pivoting is needed; a
// non-positive pivot sets bit 1 of the status word and stops.  work: r(r+1)/2 doubles, needed only
// when r exceeds SPD_REG (the triangle is kept in registers up to that order); r <= kcap.
constexpr int SPD_REG = 252;
struct SpdCholTask {
  const double* G;
  const int* rp;    // live order r
  const int* ep;    // first diagonal index that gets + 1 (null: none)
  double* C;
  int* kout;        // receives r (or the step of a breakdown)
  double* work;
  int ldg, ldc, kcap;
  int fidx;
};
// max_r: the largest kcap of the tasks (sets the launch's thread count)
void launch_spd_chol(const SpdCholTask* d_tasks, int ntasks, int max_r, int* flag, hipStream_t s);

// Leaf Cholesky Z = L L^T (lower, in place) and lower-triangular inverse.
struct LeafTask {
  double* A;
  double* B;    // the inverse of the factor (output)
  int m, lda, ldb;
  int fidx;     // status word of the owning matrix
};
// d[i] = s[i] for a list of device ints
struct IntCopy { int* d; const int* s; };
void launch_copy_ints(const IntCopy* d_list, int n, hipStream_t s);

// Band -> HODLR of X0 = (A - shift I) / scale.
struct BandDesc {
  const double* ab;
  int64_t n, ldab;
  int b;
  double shift, inv_scale;
};

// max_splits: largest GemmTask::splits among the tasks (1 when none has a workspace).
void launch_gemm(const GemmTask* d_tasks, int ntasks, int max_m, int max_n, bool fp32, hipStream_t s,
                 int max_splits = 1);
void launch_stack(const StackTask* d_tasks, int ntasks, int max_rows, int* flag, hipStream_t s);
// Stage `stage` of the TSQR of every task; a task's last stage (ceil(log2 ntiles)) also writes its R.
void launch_qr_stage(const QrTask* d_tasks, int ntasks, int stage, int max_pairs, int* flag, bool fp32,
                     hipStream_t s);
void launch_svd(const SvdTask* d_tasks, int ntasks, int* flag, bool fp32, hipStream_t s);
// fused: A (m <= 128) -> Cholesky factor, B = its inverse; whole tile in LDS
void launch_chol_inv(const LeafTask* d_tasks, int ntasks, int max_m, int* flag, hipStream_t s);
// leaves: out = alpha*X + beta*op(X)^T + gamma*I over m x m tiles (symmetrise / identity shifts)
struct LeafAxpy {
  double* out;
  const double* X;
  const double* Y;
  int m, ldo, ldx, ldy;
  int transY;
  double alpha, beta, gamma;
};
void launch_leaf_axpy(const LeafAxpy* d_tasks, int ntasks, int max_m, hipStream_t s);
void launch_fill_int(int* p, int value, int count, hipStream_t s);
void launch_copy_int(int* dst, const int* src, int count, hipStream_t s);
void launch_band_leaves(BandDesc bd, double* leaves, int ldl, const int64_t* d_leaf_lo, const int* d_leaf_m,
                        int nleaves, hipStream_t s);
struct BandBlockTask {
  double* Ul;     // rows b (lower block), ld ldu
  double* Vl;
  double* Uu;
  double* Vu;
  int* rank_l;
  int* rank_u;
  int64_t mid;
  int rows_b, rows_a, ldf;
};
void launch_band_blocks(BandDesc bd, const BandBlockTask* d_tasks, int ntasks, int max_rows, hipStream_t s);
// max over per-task ints (stats)
void launch_scale_cols(double* p, int ld, int rows, const int* wp, double scale, hipStream_t s);

}  // namespace hq

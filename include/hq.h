/*
 * hq.h -- spectral projectors of symmetric banded matrices by QDWH in HODLR format, on one AMD
 * Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * Problem (Sec. 1 of Kressner & Susnjara, "Fast computation of spectral projectors of banded
 * matrices"): for a symmetric b-banded A of order n and a shift mu with
 * lambda_nu < mu < lambda_{nu+1}, compute Pi_{<mu}(A), the orthogonal projector onto the
 * eigenvectors of the nu eigenvalues below mu, as Pi = (I - sign(A - mu I)) / 2 (Sec. 2).  The sign
 * function is the limit of the QDWH iteration (eq. reccur, weights eq. qdwh_parameters_abc); the
 * first step uses the structured QR of Sec. 4 (Algorithms 1/2), every later step the Cholesky form
 * (eq. qdwh_chol_reccur), all in HODLR format (Sec. 3.1.1) -- Algorithm hQDWH (Sec. 5).
 *
 * Conventions
 *  - Band input: LAPACK lower band storage, column-major, ab[i + j*ldab] = A(j+i, j) for
 *    0 <= i <= b, ldab >= b+1; only the lower triangle is read (A is symmetric by construction).
 *  - Pointers documented "device" are HIP device pointers; "host" are ordinary host pointers.
 *    Inputs are borrowed: they must stay valid until the call's work has completed on `stream`.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Every call returns hq_status; 0 is success.  No C++ exception crosses the ABI.  On error the
 *    output handle is set to NULL.  hq_last_error() gives a message for the calling thread.
 *  - A handle owns all device memory of its HODLR matrix until hodlr_destroy.  Calls on one handle
 *    are not reentrant: issue them from one thread, in order.
 */
#ifndef HQ_H
#define HQ_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HQ_OK = 0,
  HQ_ERR_ARG = -1,            /* invalid argument; hq_last_error() names it */
  HQ_ERR_ALLOC = -2,          /* device or host allocation failed */
  HQ_ERR_DEVICE = -3,         /* HIP runtime error */
  HQ_ERR_UNSUPPORTED = -4,    /* e.g. bandwidth larger than the smallest diagonal block */
  HQ_ERR_SINGULAR_SHIFT = 1,  /* mu is (numerically) an eigenvalue: no positive lower bound l0 */
  HQ_ERR_NOT_POSDEF = 2,      /* a leaf of Z = I + c X^T X lost positive definiteness */
  HQ_ERR_NO_CONVERGENCE = 3,  /* |1 - l_k| > delta after max_iter steps of the weight recurrence */
  HQ_ERR_RANK_OVERFLOW = 4,   /* an off-diagonal rank exceeded opts.max_rank even after regrowth */
  HQ_ERR_NONFINITE = 5        /* a non-finite value appeared in a recompression (result discarded) */
} hq_status;

typedef struct hq_hodlr_s* hq_hodlr_t;         /* opaque HODLR matrix on the device */
typedef struct hq_predictor_s* hq_predictor_t; /* opaque rank predictor (see below) */
typedef struct hq_hmatrix_s* hq_hmatrix_t;     /* opaque H-matrix (Sec. 3.1.2) on the device */

typedef struct {
  int32_t leaf;      /* n_min: diagonal blocks have at most this many rows (Alg. 3 input), >= 2 */
  double tol;        /* epsilon: absolute truncation tolerance of every recompression (Sec. 5), > 0 */
  double delta;      /* stopping tolerance |1 - l_k| <= delta (Alg. 3), default 1e-15 */
  int32_t max_rank;  /* largest off-diagonal rank a block may reach, default 512 */
  int32_t max_iter;  /* bound on QDWH iterations, default 10 */
  int32_t record_ranks;      /* nonzero: fill hq_info.level_ranks (one extra readback per iteration) */
  hq_predictor_t predictor;  /* NULL: capacities of iteration k from the ranks of X_k (2r + 16);
                                else the predictor's ranks (no readback of ranks between iterations) */
  int32_t precision;         /* HQ_FP64 (default) or HQ_MIXED */
  double c_fp32_max;         /* HQ_MIXED: a Cholesky iteration k >= 1 that is not the last and has
                                c_k <= c_fp32_max runs its GEMMs, TSQRs and core SVDs in FP32 (FP32
                                MFMA, truncation at max(tol, 8 u32 sigma_1)); default 16.  Leaf
                                Cholesky factorisations, the first and last iterations and the
                                symmetrisation stay FP64 (so Z = I + c X^T X, with condition number
                                up to 1 + c, is only formed in FP32 when c is moderate). */
  int32_t graph;             /* nonzero: capture each Cholesky iteration (k >= 1: the product for Z,
                                the H-Cholesky, the two products of the solves, all streams) into one
                                HIP graph and launch it as a whole.  Currently disabled: a nonzero
                                value returns HQ_ERR_UNSUPPORTED.  Default 0 (launches one by one). */
  int32_t method;            /* HQ_METHOD_QDWH (default): Alg. 3.  HQ_METHOD_ZOLO: Zolo-pd, the
                                polar decomposition by Zolotarev's rational functions that Sec. 2.1
                                cites (Nakatsukasa and Freund, SIAM Review 58, 2016): each step maps
                                X to mhat (X + sum_{j=1..r} a_j X (X^T X + c_{2j-1} I)^{-1}), about
                                two steps in all; the first step takes r structured QR factorisations
                                of [X_0; sqrt(c_{2j-1}) I] (Algorithms 1/2), the later ones r
                                H-Cholesky factorisations of X^T X + c_{2j-1} I issued as one batch.
                                FP64 only (precision and predictor are ignored); batched calls advance
                                their members together, each with its own degree and schedule. */
  int32_t zolo_r;            /* HQ_METHOD_ZOLO: the degree r in [1, 8]; 0 (default) picks the smallest
                                r reaching |1 - l_K| <= delta in two steps (r = 8 and more steps when
                                none does) */
} hq_opts;
#define HQ_METHOD_QDWH 0
#define HQ_METHOD_ZOLO 1
#define HQ_FP64 0
#define HQ_MIXED 1

typedef struct {
  int32_t iters;             /* QDWH iterations K (Zolo-pd: its steps; then a[k] holds mhat_k, b[k]
                                the lower bound l_k, c[k] the smallest shift c_1 of step k) */
  double alpha;              /* scaling alpha >= ||A - mu I||_2 */
  double l0;                 /* certified lower bound of sigma_min((A - mu I)/alpha) */
  double a[16], b[16], c[16];/* weights of each iteration */
  int32_t max_rank_iter[16]; /* largest off-diagonal rank of X_{k+1} */
  int32_t max_rank;          /* largest off-diagonal rank of the returned matrix */
  int32_t redo_count;        /* iterations repeated after a capacity overflow */
  int64_t bytes;             /* device bytes of the returned matrix */
  int64_t peak_bytes;        /* peak device working set of the solve */
  int64_t launches;          /* kernel launches issued */
  double seconds;            /* wall time of the call */
  double setup_seconds;      /* alpha, l0 and the weight schedule (host) */
  double givens_seconds;     /* Algorithms 1/2 and the Q factors (host) */
  int32_t levels;            /* tree depth L */
  /* opts.record_ranks: largest rank at level l (< 24) of the outputs of iteration k (< 16):
   * [k][0] X_{k+1}, and for k >= 1 [k][1] Z_k = I + c X^T X, [k][2] L_k^{-1}, [k][3] Y_k */
  int32_t level_ranks[16][4][24];
  int64_t capacity_columns;  /* sum over iterations of the factor columns allocated for X_{k+1}, Z, L, Y */
  int32_t fp32_iter[16];     /* 1 where iteration k ran in FP32 (HQ_MIXED) */
  int32_t graphs;            /* opts.graph: iterations launched as captured graphs */
  int64_t graph_nodes;       /* opts.graph: kernel and dependency nodes in those graphs */
  double graph_build_seconds;/* opts.graph: host time spent capturing and instantiating them */
  int32_t zolo_r;            /* HQ_METHOD_ZOLO: the degree r used (0 for QDWH) */
  double iter_seconds[16];   /* wall time of iteration k (Zolo-pd: step k), host work of k = 0 and
                                repeats after a capacity overflow included, up to its rank readback */
} hq_info;

/* Fill *o with the defaults: leaf 256, tol 1e-10, delta 1e-15, max_rank 512, max_iter 10. */
hq_status hq_default_opts(hq_opts* o);

/*
 * X0 = (A - shift I) / scale as an exact HODLR matrix (Alg. 3, X_0 = A/alpha with the shift of
 * Sec. 2).  band: device.  Every off-diagonal block is the b x b corner next to the diagonal, stored
 * with rank b; requires b <= the smallest diagonal block.  Stream-ordered, asynchronous.
 */
hq_status hodlr_build(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                      const hq_opts* opts, void* stream, hq_hodlr_t* out);

/*
 * Solve H X = B for a symmetric positive definite HODLR matrix H (for instance hodlr_build of an SPD
 * band; the lower blocks are read): the H-Cholesky H = L L^T of Alg. 3 (truncation at tol), then
 *   method 0: the HODLR triangular solves of Table complexity_HODLR by substitution over the tree
 *             (L T = B, then L^T X = T: one leaf product and two thin products per block, depth first);
 *   method 1: the products with L^{-1} that the factorisation also forms, X = L^{-T} (L^{-1} B), the
 *             route the QDWH iteration takes (level-parallel launches).
 * B and X: device, n x ncols, column-major (ldb, ldx >= n); B is not modified.  cap: rank capacity of
 * the inverse blocks (0: 64; HQ_ERR_RANK_OVERFLOW above it).  seconds (host, may be NULL) receives
 * the wall times [factorisation, solve].  Blocks until done.  HQ_ERR_NOT_POSDEF if H is not.
 */
hq_status hodlr_cholesky_solve(hq_hodlr_t H, const double* B, int64_t ldb, int32_t ncols, double* X, int64_t ldx,
                               double tol, int32_t cap, int32_t method, void* stream, double* seconds);

/*
 * U ~ sign(A - mu I) in HODLR format (Sec. 2; Alg. 3 lines up to "U = X_k", symmetrised).
 * band: device.  Blocks until done (returns host status and info).  info may be NULL.
 */
hq_status qdwh_sign(const double* band, int64_t n, int32_t b, int64_t ldab, double mu, const hq_opts* opts,
                    void* stream, hq_hodlr_t* sign_out, hq_info* info);

/*
 * P ~ Pi_{<mu}(A) = (I - sign(A - mu I)) / 2 in HODLR format (Alg. 3, output P).  band: device.
 * Blocks until done.  info may be NULL.
 */
hq_status spectral_projector(const double* band, int64_t n, int32_t b, int64_t ldab, double mu,
                             const hq_opts* opts, void* stream, hq_hodlr_t* P_out, hq_info* info);

/*
 * Batched form of spectral_projector for `count` independent problems (Alg. 3 for each member),
 * 1 <= count <= 1024.  bands[i]: device band of member i; n, b, ldab, mu: host arrays of `count`
 * entries.  The members advance together: every kernel launch of a step serves all members still
 * iterating, so many small or uneven problems fill the device.  P_out[i] receives member i's
 * projector (NULL if that member failed); info (may be NULL) receives `count` records whose
 * seconds, launches and peak_bytes describe the whole batch.  Returns HQ_OK when every member
 * succeeded, otherwise the status of the first member that failed (the others are still
 * computed and returned).  Blocks until done.
 */
hq_status spectral_projector_batched(int32_t count, const double* const* bands, const int64_t* n, const int32_t* b,
                                     const int64_t* ldab, const double* mu, const hq_opts* opts, void* stream,
                                     hq_hodlr_t* P_out, hq_info* info);

/*
 * Y = P X for a HODLR matrix P (Table complexity_HODLR, matrix-vector product, O(k n log n) per
 * column).  X: device, n x ncols, column-major, ldx >= n.  Y: device, ldy >= n, overwritten; must
 * not overlap X.  Stream-ordered, asynchronous.
 */
hq_status apply_projector(hq_hodlr_t P, const double* X, int64_t ldx, int32_t ncols, double* Y, int64_t ldy,
                          void* stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same product Y = P X as apply_projector, with the same kernels and
 * arguments, but its device workspace comes from one static device array per GPU
 * (apply_projector_noalloc_max_bytes() bytes, 64 MiB, held until the process ends) and its task
 * descriptors from pinned memory the handle reserved when it was made; no device or pinned memory is
 * allocated or freed.  A call whose workspace would exceed the maximum (it grows with ncols and the
 * ranks of P) returns HQ_ERR_ARG before launching anything.  Every call on a GPU uses that GPU's one
 * array, which keeps the last call's contents: calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  Like apply_projector, a call waits on the host
 * until the previous apply of the same handle has read its descriptors.  Stream-ordered otherwise.
 */
hq_status apply_projector_noalloc(hq_hodlr_t P, const double* X, int64_t ldx, int32_t ncols, double* Y,
                                  int64_t ldy, void* stream);
size_t apply_projector_noalloc_max_bytes(void);

/* Dense copy (device, n x n, ld >= n) of a HODLR matrix; meant for tests and small n. */
hq_status hodlr_to_dense(hq_hodlr_t H, double* out, int64_t ld, void* stream);

/* Structure of a handle: order, tree levels, number of leaves, sum of leaf traces (host values). */
hq_status hodlr_shape(hq_hodlr_t H, int64_t* n, int32_t* levels, int32_t* nleaves, int32_t* max_rank);
/* Host copy of leaf i: rows/cols [*lo, *lo + *m); out: host, ld >= m. */
hq_status hodlr_get_leaf(hq_hodlr_t H, int32_t i, double* out, int64_t ld, int64_t* lo, int64_t* m);
/* Host copy of off-diagonal block `which` (0 upper, 1 lower) of internal node `node` (heap order):
 * U: rows x rank, V: cols x rank (ld >= rows/cols, capacity >= *rank).  Pass U = V = NULL to query
 * rank and extents only.  lo/mid/hi give the node's row range and split. */
hq_status hodlr_get_block(hq_hodlr_t H, int32_t node, int32_t which, double* U, double* V, int64_t ld,
                          int32_t* rank, int64_t* lo, int64_t* mid, int64_t* hi);

/*
 * mu between lambda_nu and lambda_{nu+1}: the midpoint, by Sylvester-inertia bisection on the host
 * (band: host).  Also returns the gap lambda_{nu+1} - lambda_nu.  1 <= nu < n.
 */
hq_status hq_shift_for_count(const double* band, int64_t n, int32_t b, int64_t ldab, int64_t nu, double* mu,
                             double* gap);

void hodlr_destroy(hq_hodlr_t H);
const char* hq_status_string(hq_status s);
const char* hq_last_error(void);

/*
 * Tile shapes and thresholds of the kernels, picked by the project's autotuner
 * (paper_1608_01164_amd/autotune.py, outside any timed region) and read by the library at first use
 * from tuning.txt next to it (or the file named by the environment variable HQ_TUNING); built-in
 * defaults when there is none.  They change how work is tiled (so results can differ in the last
 * bits between tables), never what is computed.
 *   qr_tile_rows  rows of a TSQR row tile (stage 0 of the R-only TSQR of the recompressions), 32..8192
 *   split_min_k   GEMMs with an inner dimension >= this split it over workgroups, >= 64
 *   split_chunk   rows of the inner dimension per split, >= 32
 *   split_max     most splits, 1..128
 *   schur_keep    the H-Cholesky carries its lazy Schur factor uncompressed up to this many columns
 *   gemm_small_tiles  batched GEMM launches of at most this many 64 x 64 output tiles (inner dimension
 *                 not split) run with 32 x 32 tiles and register-staged operands, 0..2^20 (0: never);
 *                 both kernels give the same result bit for bit
 * hq_tuning_set replaces the table for the rest of the process (all values checked, HQ_ERR_ARG if out
 * of range); it must not be called while a solve runs.  hq_tuning_source names where the values came
 * from.
 */
typedef struct { int32_t qr_tile_rows, split_min_k, split_chunk, split_max, schur_keep, gemm_small_tiles; } hq_tuning;
hq_status hq_tuning_get(hq_tuning* out);
hq_status hq_tuning_set(const hq_tuning* in);
const char* hq_tuning_source(void);

/* ---- Test hooks: single building blocks of the path, exposed so that tests can compare each one
 *      with an independent reference.  All pointers device unless stated. ---- */
/* fp32 != 0 selects the FP32 variant of a kernel (operands rounded to FP32, FP32 arithmetic; inputs
 * and outputs stay FP64 in memory), as used by the middle iterations of the mixed precision mode. */
/* C = alpha op(A) op(B) + beta C through the batched MFMA GEMM kernel. */
hq_status hq_test_gemm(const double* A, const double* B, double* C, int32_t m, int32_t n, int32_t k,
                       int32_t lda, int32_t ldb, int32_t ldc, int32_t opA, int32_t opB, double alpha, double beta,
                       int32_t fp32, void* stream);
/* R factor (r x r, upper, ldr = r) of the Householder TSQR of M (rows x r). */
hq_status hq_test_qr_r(const double* M, int32_t rows, int32_t r, int32_t ldm, double* R, int32_t fp32, void* stream);
/* Truncated recompression of Us (m x r) Vs^T (n x r): U (m x k), V (n x k), *k host. */
hq_status hq_test_recompress(const double* Us, int32_t m, const double* Vs, int32_t n, int32_t r, double tol,
                             int32_t kcap, double* U, double* V, int32_t* k, int32_t fp32, void* stream);
/* HODLR approximation of a dense symmetric-or-not matrix (device, n x n, ld) by truncated SVD of
 * every off-diagonal block. */
hq_status hq_test_from_dense(const double* dense, int64_t n, int64_t ld, const hq_opts* opts, int32_t cap,
                             void* stream, hq_hodlr_t* out);
/* C = alpha op(A) op(B) + delta * (D or I); lower_only keeps the lower blocks only (symmetric C). */
hq_status hq_test_product(hq_hodlr_t A, int32_t transA, hq_hodlr_t B, int32_t transB, double alpha, hq_hodlr_t D,
                          int32_t d_identity, double delta, int32_t lower_only, int32_t cap, double tol,
                          void* stream, hq_hodlr_t* out);
/* L^{-1} of the Cholesky factor of a symmetric positive definite HODLR Z (lower blocks used). */
hq_status hq_test_cholesky_inverse(hq_hodlr_t Z, int32_t cap, double tol, void* stream, hq_hodlr_t* out);
/* Q1, Q2 of the structured QR of [scale*(A - shift I); I] (band: host) in HODLR format. */
hq_status hq_test_q_factors(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                            int32_t leaf, void* stream, hq_hodlr_t* q1, hq_hodlr_t* q2, int64_t* nrot);

/*
 * Rank predictor: a perceptron (10 inputs, two tanh layers of 32, 4 linear outputs; FP32) that maps
 * (level, block size, bandwidth, iteration, weights c_k and a_k, rank of X_k at the level, l0, n,
 * tol) to the codes log2(1 + r)/10 of the largest ranks at that level of X_{k+1}, Z_k, L_k^{-1}
 * and Y_k.  Used through opts.predictor, it sets every capacity before the iterations start;
 * a rank above its capacity is caught by the kernels and the iteration is repeated with larger
 * capacities, so results do not depend on the predictions.  Training and inference run in the
 * library's own kernels.  Parameters: W1 (32x10), b1, W2 (32x32), b2, W3 (4x32), b3, row-major.
 */
#define HQ_PRED_FEATURES 10
#define HQ_PRED_OUTPUTS 4
/* New network with Glorot-uniform weights from `seed` (splitmix64), zero biases. */
hq_status hq_predictor_create(uint64_t seed, hq_predictor_t* out);
int64_t hq_predictor_nparams(void);
/* Host copies of the parameters (nparams floats). */
hq_status hq_predictor_get_params(hq_predictor_t p, float* params);
hq_status hq_predictor_set_params(hq_predictor_t p, const float* params);
/* Safety margins (4 floats in [0, 1], host), added to the predicted codes before they become
 * capacities: capacity = 2^(10 (code + margin)) - 1 + 4.  Default 0.05 each. */
hq_status hq_predictor_set_margin(hq_predictor_t p, const float* margin);
hq_status hq_predictor_get_margin(hq_predictor_t p, float* margin);
/* Y = net(X): X device rows x 10, Y device rows x 4, row-major.  Stream-ordered. */
hq_status hq_predictor_forward(hq_predictor_t p, const float* X, int64_t rows, float* Y, void* stream);
/* Loss sum w (y - t)^2 / sum w over rows (X, T, W device, row-major) and its gradient (device,
 * nparams floats).  *loss: host.  Blocks until done. */
hq_status hq_predictor_loss_grad(hq_predictor_t p, const float* X, const float* T, const float* W, int64_t rows,
                                 float* loss, float* grad, void* stream);
/* `epochs` full-batch Adam steps (learning rate lr); *loss: host, the loss before the last step. */
hq_status hq_predictor_train(hq_predictor_t p, const float* X, const float* T, const float* W, int64_t rows,
                             int32_t epochs, float lr, void* stream, float* loss);
/* Training rows from a solve run with opts.record_ranks (host outputs, up to 16*24 rows each of
 * X (10 floats), T and W (4 floats); W masks entries that do not exist).  The features are built
 * by the same code the solver uses, with the recorded rank of X_k as the previous rank. */
hq_status hq_predictor_rows(const hq_info* info, int64_t n, int32_t b, const hq_opts* opts, float* X, float* T,
                            float* W, int32_t* rows);
void hq_predictor_destroy(hq_predictor_t p);

/* Built-in kernel timers: when enabled, every launch of the library is bracketed by HIP events on
 * its own stream and the kernels count their algorithmic work (flops, operand bytes).
 * hq_profile_read synchronises the device and returns, per kernel class (0 gemm, 1 tsqr, 2 core svd,
 * 3 leaf cholesky, 4 leaf inverse, 5 stack, 6 leaf elementwise, 7 other), the number of launches,
 * total milliseconds, flops and bytes since the last reset; reset != 0 clears them. */
typedef struct { int64_t launches; double ms, flops, bytes; } hq_kstat;
hq_status hq_profile_enable(int32_t on);
/* Restricts the timers to the classes in mask (bit c for class c; -1, the initial value, times all):
 * launches of other classes get no events, so a run that needs one class's durations pays for no
 * others.  The kernels' work counters run for every class while profiling is on. */
hq_status hq_profile_select(int32_t mask);
hq_status hq_profile_read(hq_kstat* out /* [8] */, int32_t reset);
/* Flops the kernels issued as MFMA instructions since the last reset (counted while profiling is on):
 * out[0] FP64, out[1] FP32 (host); reset != 0 clears them.  Synchronises the device. */
hq_status hq_profile_mfma(double* out /* [2] */, int32_t reset);
/* Core-SVD internals since the last reset: [0..2] cycles of the pivoted-QR, Jacobi and output phases
 * (wall clock at 100 MHz), [3] sum of r, [4] sum of t, [5] sum of sweeps, [6] cores. */
hq_status hq_profile_svd(int64_t* out /* [8] */);

/* Sec. 3.1.2 (eq. stand_adm) and Example hodlrvshmatrix: the H-matrix form of a HODLR matrix P (for
 * instance a projector from spectral_projector), for the partition of the HODLR cluster tree in which
 * a block t x s of two clusters of one level is admissible iff min(diam t, diam s) <= dist(t, s)
 * (diam t = max |i - j| over t, dist(t, s) = min |i - j|, i in t, j in s), the recursion over the
 * children pairs stopping at an admissible block (stored as U V^T) or at a leaf cluster (stored
 * dense).  Every admissible sub-block of a HODLR off-diagonal block is recompressed on its own at the
 * absolute tolerance tol (> 0; opts.tol of the solve is the natural choice); the dense blocks are the
 * HODLR leaves and one corner per off-diagonal block next to the diagonal.  P must outlive the result
 * (its diagonal blocks are shared).  Runs on `stream` and returns with it synchronised.  Errors:
 * HQ_ERR_ARG (NULL handle or output, tol <= 0), HQ_ERR_NONFINITE (a sub-block recompression met
 * non-finite values). */
hq_status hodlr_to_hmatrix(hq_hodlr_t P, double tol, void* stream, hq_hmatrix_t* out);
/* Counts and storage of an H-matrix (host outputs, each may be NULL): *n; *nlr low-rank and *ndense
 * dense blocks; *bytes = 8 x (sum over low-rank blocks of (rows + cols) x rank + sum over dense blocks
 * of rows x cols) with the blocks' actual ranks, and *hodlr_bytes the same count for the HODLR matrix
 * it was made from (off-diagonal blocks with their ranks, plus the leaves): the two columns of Table
 * storage_spec; *max_rank the largest rank of a low-rank block. */
hq_status hmatrix_shape(hq_hmatrix_t H, int64_t* n, int64_t* nlr, int64_t* ndense, int64_t* bytes,
                        int64_t* hodlr_bytes, int32_t* max_rank);
/* Block i to host memory: 0 <= i < nlr are the low-rank blocks, nlr <= i < nlr + ndense the dense ones.
 * *row0, *col0, *m, *ncols locate it; *rank is its rank (-1 for a dense block).  A low-rank block writes
 * U (m x rank) and V (ncols x rank), a dense block itself into U (m x ncols) (V unused, may be NULL);
 * column-major, leading dimension ld >= max(m, ncols).  U = NULL returns the sizes only.  Synchronous. */
hq_status hmatrix_get_block(hq_hmatrix_t H, int64_t i, int64_t* row0, int64_t* col0, int64_t* m, int64_t* ncols,
                            int32_t* rank, double* U, double* V, int64_t ld);
void hmatrix_destroy(hq_hmatrix_t H);

/* Host-only: the library's QDWH weight schedule (eq. qdwh_parameters_abc and the l_k recurrence of
 * Sec. 2.1) from a lower bound l0 in (0, 1]: a_k = h(l_k), b_k = (a_k - 1)^2 / 4, c_k = a_k + b_k - 1,
 * l_{k+1} = l_k (a_k + b_k l_k^2) / (1 + c_k l_k^2), until |1 - l_k| <= delta or max_iter (<= 16)
 * steps.  a, b, c: host, >= max_iter entries; l: host, >= max_iter + 1 entries (l_0 .. l_K); *K: host.
 * The same routine sets the schedule of every solve; no device use. */
hq_status hq_test_schedule(double l0, double delta, int32_t max_iter, double* a, double* b, double* c, double* l,
                           int32_t* K);

/* Host-only: the same Q1, Q2 assembled densely (Q1, Q2: host, n x n, ld n).  No device use. */
/* Host-only: the library's Zolo-pd coefficients of one step (see hq_opts.method) for the lower bound
 * l in [1e-150, 1) and r in [1, 16]: c[1..2r] (c_i = l^2 sc^2(i K'/(2r+1); l'), l' = sqrt(1 - l^2)),
 * a[1..r] (partial-fraction residues), *mhat = prod_j (1 + c_{2j-1})/(1 + c_{2j}) and *lnext = Zhat(l).
 * c: host, >= 2r + 1 entries; a: host, >= r + 1 entries (index 0 set to 0).  No device use. */
hq_status hq_test_zolo(double l, int32_t r, double* c, double* a, double* mhat, double* lnext);

hq_status hq_test_q_dense_host(const double* band, int64_t n, int32_t b, int64_t ldab, double shift, double scale,
                               int32_t leaf, double* Q1, double* Q2, int64_t* nrot);

#ifdef __cplusplus
}
#endif
#endif

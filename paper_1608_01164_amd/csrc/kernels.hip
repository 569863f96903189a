// Device kernels of the HODLR-QDWH path, written for CDNA4 (gfx950): 64-wide wavefronts,
// FP64 MFMA (v_mfma_f64_16x16x4f64), LDS staging.  All kernels are batched over a task array and
// read live sizes (ranks) from device memory, so a whole QDWH iteration can be issued without a
// device-to-host synchronisation.
#include "kernels.h"

#include <cfloat>
#include <cmath>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

namespace hq {

// ---------------------------------------------------------------------------------------------
// Timers and work counters
// ---------------------------------------------------------------------------------------------
__device__ unsigned long long g_prof[2 * K_NCLASS];  // [flops..., bytes...]
__device__ unsigned long long g_svdstat[8];  // phase cycles (qr, jacobi, out), sum r, sum t, sum sweeps, calls
__device__ int g_prof_on;
__device__ unsigned long long g_mfma[2];  // flops issued to the matrix cores: [0] FP64, [1] FP32

namespace {
struct Rec { hipEvent_t a, b; int cls; };
std::mutex g_mu;
bool g_on = false;
unsigned g_mask = ~0u;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}
}  // namespace

void prof_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
  const int v = on ? 1 : 0;
  (void)hipMemcpyToSymbol(HIP_SYMBOL(g_prof_on), &v, sizeof(int));
}
void prof_select(unsigned mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mask = mask;
}
bool prof_enabled() { return g_on; }
int prof_begin(int cls, hipStream_t s) {
  if (!g_on || !((g_mask >> cls) & 1u)) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{take_event(), take_event(), cls};
  (void)hipEventRecord(r.a, s);
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}
void prof_end(int slot, hipStream_t s) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(g_recs[slot].b, s);
}
void prof_svd_stats(unsigned long long out[8]) {
  (void)hipDeviceSynchronize();
  (void)hipMemcpyFromSymbol(out, HIP_SYMBOL(g_svdstat), sizeof(unsigned long long) * 8);
}
void prof_mfma(double out[2], bool reset) {
  (void)hipDeviceSynchronize();
  unsigned long long h[2];
  (void)hipMemcpyFromSymbol(h, HIP_SYMBOL(g_mfma), sizeof(h));
  out[0] = (double)h[0];
  out[1] = (double)h[1];
  if (reset) {
    unsigned long long z[2] = {0, 0};
    (void)hipMemcpyToSymbol(HIP_SYMBOL(g_mfma), z, sizeof(z));
  }
}
void prof_read(ProfStat out[K_NCLASS], bool reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  for (int c = 0; c < K_NCLASS; ++c) out[c] = ProfStat{0, 0.0, 0.0, 0.0};
  for (Rec& r : g_recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    out[r.cls].launches += 1;
    out[r.cls].ms += ms;
  }
  unsigned long long h[2 * K_NCLASS];
  (void)hipMemcpyFromSymbol(h, HIP_SYMBOL(g_prof), sizeof(h));
  for (int c = 0; c < K_NCLASS; ++c) {
    out[c].flops = (double)h[c];
    out[c].bytes = (double)h[K_NCLASS + c];
  }
  if (reset) {
    for (Rec& r : g_recs) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
    g_recs.clear();
    unsigned long long z[2 * K_NCLASS] = {};
    (void)hipMemcpyToSymbol(HIP_SYMBOL(g_prof), z, sizeof(z));
    (void)hipMemcpyToSymbol(HIP_SYMBOL(g_svdstat), z, sizeof(unsigned long long) * 8);
  }
}

static __device__ __forceinline__ void count_work(int cls, unsigned long long flops, unsigned long long bytes) {
  if (g_prof_on) {
    atomicAdd(&g_prof[cls], flops);
    if (bytes) atomicAdd(&g_prof[K_NCLASS + cls], bytes);
  }
}
// Flops a kernel issued as MFMA instructions (precision 0 FP64, 1 FP32), for the matrix-core utilisation.
static __device__ __forceinline__ void count_mfma(int prec, unsigned long long flops) {
  if (g_prof_on) atomicAdd(&g_mfma[prec], flops);
}

// A launch that the runtime rejects (resources, dimensions) must not pass silently: later kernels
// would read outputs that were never written.
static void check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

// Static plus dynamic LDS of a kernel must fit the 160 KiB of a workgroup; a dispatch above it is
// only rejected by the queue, after the launch call has returned.  Checked once per kernel.
static void check_lds(const void* kernel, size_t dynamic_bytes, const char* what) {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, kernel) != hipSuccess)
    throw std::runtime_error(std::string("cannot read the attributes of ") + what);
  if (a.sharedSizeBytes + dynamic_bytes > 160 * 1024)
    throw std::runtime_error(std::string(what) + ": static LDS " + std::to_string(a.sharedSizeBytes) + " + dynamic " +
                             std::to_string(dynamic_bytes) + " bytes exceed 160 KiB");
}

#define HQ_TIMED(cls, stream, ...)            \
  do {                                        \
    const int slot_ = prof_begin(cls, stream); \
    __VA_ARGS__;                              \
    check_launch(#cls);                       \
    prof_end(slot_, stream);                  \
  } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));

// A value every lane of the wave holds, as the compiler's scalar (wave-uniform) value: control flow
// that depends on it becomes scalar branches instead of lane masks.
static __device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads() it does not wait for this
// thread's outstanding global loads and stores, so loads issued ahead (prefetch) stay in flight and
// stores drain in the background.  For loops whose threads exchange data through LDS alone (no
// thread reads global memory another thread of the workgroup wrote during the kernel).
static __device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Live size of a task: the device count behind p (a per-task value), capped by the static bound v.
static __device__ __forceinline__ int live(const int* p, int v) {
  if (!p) return v;
  const int x = *p;
  return uniform(x < v ? x : v);
}

// Data-parallel-primitive move of a double (two 32-bit DPP moves); rows/banks masked off read 0.
template <int CTRL, int ROWS = 0xF>
static __device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Quad swaps, then rotations inside each
// 16-lane row give every lane its row sum; row broadcasts 15 and 31 fold the rows into lane 63.
static __device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);       // row_ror:4
  v += dpp_move<0x128>(v);       // row_ror:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// The same for a float (one 32-bit DPP move per step).
template <int CTRL, int ROWS = 0xF>
static __device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
static __device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x128>(v);
  v += dpp_move<0x142, 0xA>(v);
  v += dpp_move<0x143, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over a group of 16 consecutive lanes (one DPP row), returned to every lane of the group:
// quad swaps, then the half-row mirror (lane i <-> 7 - i) and the row mirror (lane i <-> 15 - i).
// Every step is a permutation inside the row, so every lane ends with the same value.  Call with
// all lanes of the wave active.
static __device__ __forceinline__ double row_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}
static __device__ __forceinline__ float row_sum(float v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return v;
}

// Precision traits of the recompression kernels.
template <typename T> struct Prec;
template <> struct Prec<double> {
  static constexpr double eps = DBL_EPSILON, tiny = DBL_MIN, big = DBL_MAX;
  static constexpr double scale_below = 0x1p-800;  // squared norms below this are recomputed scaled
  static constexpr int max_shift = 1000;           // largest single power-of-two rescaling
};
template <> struct Prec<float> {
  static constexpr float eps = FLT_EPSILON, tiny = FLT_MIN, big = FLT_MAX;
  static constexpr float scale_below = 0x1p-100f;
  static constexpr int max_shift = 100;
};

// ----------------------------------------------------------------------------------------------
// Batched GEMM, 64x64 output tile per workgroup (4 waves, 32x32 each = 2x2 MFMA 16x16 tiles),
// K staged through LDS in chunks of 16, the next chunk's loads in flight during the current
// chunk's MFMAs.  A task with a split-K workspace runs its K ranges in separate workgroups
// (blockIdx.z) that write raw partial tiles; k_gemm_reduce sums them in range order.
// ----------------------------------------------------------------------------------------------
constexpr int GT = 64, GK = 16, GQ = GT * GK / 256;  // GQ: elements of each operand a thread stages per chunk

typedef float f4 __attribute__((ext_vector_type(4)));

// Staging map of the GQ elements a thread loads per chunk: (kk, i) of element q for a tile stored
// column-major (op = 0: element (i, kk), consecutive threads on consecutive rows i; op = 1: element
// (kk, i), consecutive threads on consecutive kk).
static __device__ __forceinline__ int stage_kk(int op, int tid, int q) {
  return op == 0 ? (tid / GT) + (256 / GT) * q : tid & (GK - 1);
}
static __device__ __forceinline__ int stage_i(int op, int tid, int q) {
  return op == 0 ? tid & (GT - 1) : (tid / GK) + (256 / GK) * q;
}

// T = double: FP64 MFMA 16x16x4; T = float: operands rounded to FP32, FP32 MFMA 16x16x4 with FP32
// accumulation (alpha, beta and C stay FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_gemm(const GemmTask* __restrict__ tasks, int tiles_n) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  const GemmTask Tk = tasks[blockIdx.y];
  const int m = live(Tk.mp, Tk.m), n = live(Tk.np, Tk.n), k = live(Tk.kp, Tk.k);
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int row0 = tm * GT, col0 = tn * GT;
  if (row0 >= m || col0 >= n) return;
  const int S = Tk.W ? Tk.splits : 1, z = blockIdx.z;
  if (z >= S) return;
  int kb = 0, ke = k;
  if (S > 1) {
    const int kc = ((k + S - 1) / S + GK - 1) / GK * GK;
    kb = z * kc < k ? z * kc : k;
    ke = kb + kc < k ? kb + kc : k;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  if (blockIdx.x == 0 && z == 0 && tid == 0) {
    count_work(K_GEMM, 2ull * m * n * k,
               8ull * ((unsigned long long)m * k + (unsigned long long)k * n + (Tk.beta != 0.0 ? 2ull : 1ull) * m * n));
    count_mfma(std::is_same<T, double>::value ? 0 : 1, 2ull * m * n * k);
  }

  __shared__ T As[GK][GT + 1];
  __shared__ T Bs[GK][GT + 1];

  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};

  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  T ra[GQ], rb[GQ];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
      {
        const int gi = row0 + stage_i(Tk.opA, tid, q), gk = k0 + stage_kk(Tk.opA, tid, q);
        const bool in = gi < m && gk < ke;
        ra[q] = (T)(in ? (Tk.opA == 0 ? Tk.A[gi + (size_t)gk * Tk.lda] : Tk.A[gk + (size_t)gi * Tk.lda]) : 0.0);
      }
      {
        const int ob = Tk.opB == 0 ? 1 : 0;
        const int gj = col0 + stage_i(ob, tid, q), gk = k0 + stage_kk(ob, tid, q);
        const bool in = gj < n && gk < ke;
        rb[q] = (T)(in ? (Tk.opB == 0 ? Tk.B[gk + (size_t)gj * Tk.ldb] : Tk.B[gj + (size_t)gk * Tk.ldb]) : 0.0);
      }
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
      const int ob = Tk.opB == 0 ? 1 : 0;
      As[stage_kk(Tk.opA, tid, q)][stage_i(Tk.opA, tid, q)] = ra[q];
      Bs[stage_kk(ob, tid, q)][stage_i(ob, tid, q)] = rb[q];
    }
    lds_barrier();
    if (k0 + GK < ke) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const T a0 = As[kk + lk][wr + li], a1 = As[kk + lk][wr + 16 + li];
      const T b0 = Bs[kk + lk][wc + li], b1 = Bs[kk + lk][wc + 16 + li];
      if constexpr (std::is_same<T, double>::value) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      } else {
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    lds_barrier();
  }
  // D(i, j) of a 16x16 block: FP64 in lane j + 16 (i % 4), element i / 4; FP32 in lane
  // j + 16 (i / 4), element i % 4
  double* P = nullptr;
  if (S > 1) P = Tk.W + ((size_t)(tm * ((Tk.n + GT - 1) / GT) + tn) * S + z) * (GT * GT);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ib = std::is_same<T, double>::value ? lk + 4 * e : 4 * lk + e;
        const int ti = wr + 16 * x + ib, tj = wc + 16 * y + li;
        if (P) {
          P[ti + GT * tj] = (double)acc[x][y][e];
        } else {
          const int gi = row0 + ti, gj = col0 + tj;
          if (gi < m && gj < n) {
            double* c = Tk.C + gi + (size_t)gj * Tk.ldc;
            const double v = Tk.alpha * (double)acc[x][y][e];
            *c = (Tk.beta == 0.0) ? v : v + Tk.beta * (Tk.Cin ? Tk.Cin[gi + (size_t)gj * Tk.ldcin] : *c);
          }
        }
      }
}

// C = alpha * (sum of the split-K partial tiles, in range order) + beta * C.
__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmTask* __restrict__ tasks, int tiles_n) {
  const GemmTask Tk = tasks[blockIdx.y];
  if (!Tk.W || Tk.splits <= 1) return;
  const int m = live(Tk.mp, Tk.m), n = live(Tk.np, Tk.n);
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int row0 = tm * GT, col0 = tn * GT;
  if (row0 >= m || col0 >= n) return;
  const int S = Tk.splits;
  const double* P = Tk.W + (size_t)(tm * ((Tk.n + GT - 1) / GT) + tn) * S * (GT * GT);
  for (int e = threadIdx.x; e < GT * GT; e += 256) {
    const int ti = e % GT, tj = e / GT, gi = row0 + ti, gj = col0 + tj;
    if (gi >= m || gj >= n) continue;
    double sum = 0.0;
    for (int z = 0; z < S; ++z) sum += P[(size_t)z * (GT * GT) + e];
    double* c = Tk.C + gi + (size_t)gj * Tk.ldc;
    const double v = Tk.alpha * sum;
    *c = (Tk.beta == 0.0) ? v : v + Tk.beta * (Tk.Cin ? Tk.Cin[gi + (size_t)gj * Tk.ldcin] : *c);
  }
}

// Small batched GEMMs (a launch of few output tiles, K not split): the GPU would leave most compute
// units idle under 64 x 64 tiles, and each tile would wait on one memory round trip per 16-deep K
// chunk.  Here a workgroup covers 32 x 32 outputs, each wave one 16 x 16 block, GSK deep in K at a
// time with the next chunk's loads in flight during the current chunk's MFMAs.  Lane l takes
// A(i0 + l % 16, k0 + 4 s + l / 16) and B(k0 + 4 s + l / 16, j0 + l % 16) into step s.  An operand
// whose rows run along memory (A not transposed, B transposed) is loaded in that layout directly;
// one stored K-contiguous (A^T, B) is read with consecutive lanes on consecutive K, GSK values of a
// row per instruction, and turned into the step layout through a slice of LDS that only its own
// wave touches (no workgroup barrier).  Loads are unconditional (an element outside the operand
// reads element 0 and is replaced by zero), so that a chunk's loads are all in flight together.
// A task runs 4 ceil(k / 16) steps in K order, as in k_gemm (zeros past k), so both kernels give
// the same result bit for bit.
constexpr int GS_T = 32, GSK = 64, GSS = GSK / 4, GS_LD = GSK + 1;

template <typename T, bool AKC, bool BKC>
static __device__ __forceinline__ void gemm_small_loop(const GemmTask& Tk, const int m, const int n, const int k,
                                                       const int row0, const int col0, const int lane, T* sa, T* sb,
                                                       typename std::conditional<std::is_same<T, double>::value, d4,
                                                                                 f4>::type& acc) {
  const int li = lane & 15, lk = lane >> 4;
  T ra[GSS], rb[GSS];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < GSS; ++q) {
      const int ai = AKC ? row0 + q : row0 + li, ak = AKC ? k0 + lane : k0 + 4 * q + lk;
      const bool ain = ai < m && ak < k;
      const size_t aidx = ain ? (AKC ? ak + (size_t)ai * Tk.lda : ai + (size_t)ak * Tk.lda) : 0;
      const double av = Tk.A[aidx];
      ra[q] = (T)(ain ? av : 0.0);
      const int bj = BKC ? col0 + q : col0 + li, bk = BKC ? k0 + lane : k0 + 4 * q + lk;
      const bool bin = bj < n && bk < k;
      const size_t bidx = bin ? (BKC ? bk + (size_t)bj * Tk.ldb : bj + (size_t)bk * Tk.ldb) : 0;
      const double bv = Tk.B[bidx];
      rb[q] = (T)(bin ? bv : 0.0);
    }
  };
  load(0);
  for (int k0 = 0; k0 < k; k0 += GSK) {
    T ca[GSS], cb[GSS];
    if constexpr (AKC) {
#pragma unroll
      for (int q = 0; q < GSS; ++q) sa[q * GS_LD + lane] = ra[q];
    }
    if constexpr (BKC) {
#pragma unroll
      for (int q = 0; q < GSS; ++q) sb[q * GS_LD + lane] = rb[q];
    }
    // the slices are this wave's alone and a wave's LDS accesses complete in order: only the
    // compiler must keep the reads below after the writes above
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < GSS; ++q) {
      ca[q] = AKC ? sa[li * GS_LD + 4 * q + lk] : ra[q];
      cb[q] = BKC ? sb[li * GS_LD + 4 * q + lk] : rb[q];
    }
    // and the next chunk's writes after these reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (k0 + GSK < k) load(k0 + GSK);
    const int left = k - k0;  // groups of 16 K (four steps) as k_gemm's chunks, zeros past k
#pragma unroll
    for (int g = 0; g < GSK / 16; ++g) {
      if (g * 16 >= left) break;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = 4 * g + u;
        if constexpr (std::is_same<T, double>::value)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[q], cb[q], acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[q], cb[q], acc, 0, 0, 0);
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_small(const GemmTask* __restrict__ tasks, int tiles_n) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  __shared__ T slab[4][2][16 * GS_LD];  // per wave: A rows, B columns of the current chunk
  const GemmTask Tk = tasks[blockIdx.y];
  const int m = live(Tk.mp, Tk.m), n = live(Tk.np, Tk.n), k = live(Tk.kp, Tk.k);
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  if (blockIdx.x == 0 && tid == 0) {
    count_work(K_GEMM, 2ull * m * n * k,
               8ull * ((unsigned long long)m * k + (unsigned long long)k * n + (Tk.beta != 0.0 ? 2ull : 1ull) * m * n));
    count_mfma(std::is_same<T, double>::value ? 0 : 1, 2ull * m * n * k);
  }
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int row0 = tm * GS_T + (wave >> 1) * 16, col0 = tn * GS_T + (wave & 1) * 16;
  if (row0 >= m || col0 >= n) return;  // wave-uniform: this wave's block lies outside C
  Acc acc = Acc{0, 0, 0, 0};
  if (k > 0) {
    T* const sa = slab[wave][0];
    T* const sb = slab[wave][1];
    const int akc = uniform(Tk.opA != 0), bkc = uniform(Tk.opB == 0);  // operands stored with K contiguous
    if (akc && bkc)
      gemm_small_loop<T, true, true>(Tk, m, n, k, row0, col0, lane, sa, sb, acc);
    else if (akc)
      gemm_small_loop<T, true, false>(Tk, m, n, k, row0, col0, lane, sa, sb, acc);
    else if (bkc)
      gemm_small_loop<T, false, true>(Tk, m, n, k, row0, col0, lane, sa, sb, acc);
    else
      gemm_small_loop<T, false, false>(Tk, m, n, k, row0, col0, lane, sa, sb, acc);
  }
  // D(i, j) of the 16x16 block: FP64 in lane j + 16 (i % 4), element i / 4; FP32 in lane
  // j + 16 (i / 4), element i % 4
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = row0 + (std::is_same<T, double>::value ? lk + 4 * e : 4 * lk + e), j = col0 + li;
    if (i < m && j < n) {
      double* c = Tk.C + i + (size_t)j * Tk.ldc;
      const double v = Tk.alpha * (double)acc[e];
      *c = (Tk.beta == 0.0) ? v : v + Tk.beta * (Tk.Cin ? Tk.Cin[i + (size_t)j * Tk.ldcin] : *c);
    }
  }
}

void launch_gemm(const GemmTask* d_tasks, int ntasks, int max_m, int max_n, bool fp32, hipStream_t s,
                 int max_splits) {
  if (ntasks <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = (max_m + GT - 1) / GT, tn = (max_n + GT - 1) / GT;
  const int zs = max_splits > 1 ? max_splits : 1;
  if (zs == 1 && ntasks <= 65535 && (long long)tm * tn * ntasks <= tuning().gemm_small_tiles) {
    const int sm = (max_m + GS_T - 1) / GS_T, sn = (max_n + GS_T - 1) / GS_T;
    if (fp32)
      HQ_TIMED(K_GEMM, s, hipLaunchKernelGGL(k_gemm_small<float>, dim3(sm * sn, ntasks), dim3(256), 0, s, d_tasks, sn));
    else
      HQ_TIMED(K_GEMM, s, hipLaunchKernelGGL(k_gemm_small<double>, dim3(sm * sn, ntasks), dim3(256), 0, s, d_tasks, sn));
    return;
  }
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    const int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    if (fp32)
      HQ_TIMED(K_GEMM, s, hipLaunchKernelGGL(k_gemm<float>, dim3(tm * tn, nt, zs), dim3(256), 0, s, d_tasks + t0, tn));
    else
      HQ_TIMED(K_GEMM, s, hipLaunchKernelGGL(k_gemm<double>, dim3(tm * tn, nt, zs), dim3(256), 0, s, d_tasks + t0, tn));
    if (zs > 1)
      HQ_TIMED(K_GEMM, s, hipLaunchKernelGGL(k_gemm_reduce, dim3(tm * tn, nt), dim3(256), 0, s, d_tasks + t0, tn));
  }
}

// ----------------------------------------------------------------------------------------------
// Column stacking with scaling at device-determined offsets.
// ----------------------------------------------------------------------------------------------
// A workgroup covers 64 rows and 4 column phases; blockIdx.z spreads the columns further, so that a
// stack of a few thousand rows still fills many workgroups, and each thread has four loads in flight
// before it stores.
constexpr int STK_ROWS = 64, STK_PH = 4, STK_Z = 4;
__global__ __launch_bounds__(256) void k_stack(const StackTask* __restrict__ tasks, int* flag) {
  const StackTask* T = tasks + blockIdx.y;
  const int row = blockIdx.x * STK_ROWS + (threadIdx.x & (STK_ROWS - 1));
  const int c0 = blockIdx.z * STK_PH + threadIdx.x / STK_ROWS, cs = STK_PH * gridDim.z;
  const int rows = T->rows, ld = T->ld, nsrc = T->nsrc, wcap = T->wcap;
  const bool lead = blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0;
  double* __restrict__ dst = T->dst;
  int off = 0;
  for (int s = 0; s < nsrc; ++s) {
    const double* __restrict__ p = T->src[s].p;
    const int* wp = T->src[s].wp;
    const int lds = T->src[s].ld;
    const double sc = T->src[s].scale;
    int w = wp ? *wp : T->src[s].w;
    if (off + w > wcap) {
      w = wcap - off;
      if (lead) atomicOr(flag + T->fidx, 4);
    }
    if (row < rows) {
      const double* q = p + row;
      double* d = dst + row + (size_t)off * ld;
      int c = c0;
      for (; c + 3 * cs < w; c += 4 * cs) {
        const double v0 = q[(size_t)c * lds], v1 = q[(size_t)(c + cs) * lds];
        const double v2 = q[(size_t)(c + 2 * cs) * lds], v3 = q[(size_t)(c + 3 * cs) * lds];
        d[(size_t)c * ld] = sc * v0;
        d[(size_t)(c + cs) * ld] = sc * v1;
        d[(size_t)(c + 2 * cs) * ld] = sc * v2;
        d[(size_t)(c + 3 * cs) * ld] = sc * v3;
      }
      for (; c < w; c += cs) d[(size_t)c * ld] = sc * q[(size_t)c * lds];
    }
    off += w;
  }
  if (T->wout && lead) *T->wout = off;
}

void launch_stack(const StackTask* d_tasks, int ntasks, int max_rows, int* flag, hipStream_t s) {
  if (ntasks <= 0) return;
  const int bx = max_rows > 0 ? (max_rows + STK_ROWS - 1) / STK_ROWS : 1;
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    const int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    HQ_TIMED(K_STACK, s, hipLaunchKernelGGL(k_stack, dim3(bx, nt, STK_Z), dim3(256), 0, s, d_tasks + t0, flag));
  }
}

__global__ void k_scale_cols(double* p, int ld, int rows, const int* wp, double scale) {
  const int w = *wp;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < rows * w; idx += gridDim.x * blockDim.x)
    p[(idx % rows) + (size_t)(idx / rows) * ld] *= scale;
}
void launch_scale_cols(double* p, int ld, int rows, const int* wp, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, dim3(64), dim3(256), 0, s, p, ld, rows, wp, scale);
  check_launch("scale_cols");
}

// ----------------------------------------------------------------------------------------------
// Householder triangularisation of an h x r panel (one workgroup).  The panel lives in LDS when it
// fits (QR_LDS doubles), else in its global workspace slot.  Each step needs two barriers: the
// norm of the next pivot column below the diagonal is accumulated while that column is updated.
// ----------------------------------------------------------------------------------------------
constexpr int QR_THREADS = 1024;
constexpr int QR_WAVES = QR_THREADS / 64;
constexpr int QR_RMAX = 1024;
constexpr int QR_LDS_BYTES = 153600;  // dynamic LDS of a TSQR stage: 150 KiB (160 KiB minus the static arrays)

template <typename T>
static __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide reduction (all threads of a QR_THREADS block, uniform control flow); every thread
// gets the result.
template <bool MAX, typename T>
static __device__ T block_reduce(T v, T* red) {
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < QR_WAVES; ++w) t = MAX ? fmax(t, red[w]) : t + red[w];
  __syncthreads();
  return t;
}

// Maximum over the 16 lanes of a DPP row (the permutations of row_sum).
static __device__ __forceinline__ double row_max(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x141>(v));
  v = fmax(v, dpp_move<0x140>(v));
  return v;
}
static __device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, dpp_move<0xB1>(v));
  v = fmaxf(v, dpp_move<0x4E>(v));
  v = fmaxf(v, dpp_move<0x141>(v));
  v = fmaxf(v, dpp_move<0x140>(v));
  return v;
}

// Householder triangularisation of a small row tile (h <= 16 EM rows, r <= 64 CPG columns) held in
// registers: column c belongs to the 16-lane group c % 64 (slot c / 64), its rows sl + 16 e to lane
// sl.  Step j: the wave holding column j forms the reflector from that column (fresh norm below the
// diagonal; a column near underflow is first rescaled by an exact power of two) and publishes it
// through LDS, double buffered and zero above row j; the groups holding columns right of j apply
// it.  One barrier per step, and the reflectors are not kept (R only).  R (min(h, r) x r, upper
// trapezoidal) goes to out (leading dimension ldo).  Every row reduction runs with the whole wave
// active; what a group computes for a column it does not own is discarded.
template <typename T, int EM, int CPG>
static __device__ void householder_regs(const double* src, int lds, T* out, int ldo, int h, int r, int* flag,
                                        int fidx, T* dyn) {
  // exchange buffers in the kernel's dynamic LDS: 2 x 16 EM reflector rows, then 2 factors
  T(*vbuf)[16 * EM] = reinterpret_cast<T(*)[16 * EM]>(dyn);
  T* tbuf = dyn + 2 * 16 * EM;
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6), sub = lane >> 4, sl = lane & 15;
  const int g = tid >> 4;  // group: 4 * wave + sub
  T x[CPG][EM];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < CPG; ++k)
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const int c = 64 * k + g, i = sl + 16 * e;
      double v = 0.0;
      if (c < r && i < h) v = src[i + (size_t)c * lds];
      bad |= !(fabs(v) <= DBL_MAX);
      x[k][e] = (T)v;
    }
  if (bad) atomicOr(flag + fidx, 16);  // non-finite stacked input
  const int jend = (h - 1 < r) ? h - 1 : r;
  unsigned long long flops = 0;
  for (int j = 0; j < jend; ++j) {
    const int b = j & 1, go = j & 63, kj = j >> 6;
    if (wave == (go >> 2)) {
      const bool owner = sub == (go & 3);
#pragma unroll
      for (int k = 0; k < CPG; ++k)
        if (k == kj) {  // wave-uniform
          T x0 = 0, s = 0, am = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const int i = sl + 16 * e;
            const T v = x[k][e];
            x0 += i == j ? v : (T)0;
            s += i > j ? v * v : (T)0;
            am = fmax(am, i >= j ? fabs(v) : (T)0);
          }
          x0 = row_sum(x0);
          s = row_sum(s);
          am = row_max(am);
          // near underflow: rows j.. rescaled by 2^-e (as two factors when 2^-e is not representable)
          const bool scaled = s < Prec<T>::scale_below && am > (T)0;
          T sc1 = 1, sc2 = 1, unscale = 1;
          if (scaled) {
            constexpr int M = Prec<T>::max_shift;
            const int ex = ilogb(am);
            sc1 = ldexp((T)1, -ex > M ? M : -ex);
            sc2 = ldexp((T)1, -ex > M ? -ex - M : 0);
            unscale = ldexp((T)1, ex);
          }
          T x0s = 0, ss = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const int i = sl + 16 * e;
            const T v = i >= j ? (x[k][e] * sc1) * sc2 : x[k][e];
            x0s += i == j ? v : (T)0;
            ss += i > j ? v * v : (T)0;
            if (owner) x[k][e] = v;
          }
          x0s = row_sum(x0s);
          ss = row_sum(ss);
          if (scaled) {
            x0 = x0s;
            s = ss;
          }
          T tau = 0, v0 = 0, rjj = x0 * unscale;
          if (s != (T)0) {
            const T nrm = sqrt(x0 * x0 + s);
            const T beta = x0 >= 0 ? -nrm : nrm;
            v0 = x0 - beta;
            tau = (T)1 / (nrm * (nrm + fabs(x0)));
            rjj = beta * unscale;
          }
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const int i = sl + 16 * e;
            if (owner) {
              vbuf[b][i] = i > j ? x[k][e] : (i == j ? v0 : (T)0);
              if (i == j) x[k][e] = rjj;
            }
          }
          if (owner && sl == 0) tbuf[b] = tau;
        }
    }
    __syncthreads();
    const T tau = tbuf[b];
    if (64 * (CPG - 1) + 4 * wave + 3 > j && tau != (T)0) {  // some slot of this wave right of j
      T v[EM];
#pragma unroll
      for (int e = 0; e < EM; ++e) v[e] = vbuf[b][sl + 16 * e];
#pragma unroll
      for (int k = 0; k < CPG; ++k)
        if (64 * k + 4 * wave + 3 > j && 64 * k + 4 * wave < r) {  // wave-uniform
          const int c = 64 * k + g;
          const bool act = c > j && c < r;
          T w = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) w += v[e] * x[k][e];
          w = row_sum(w) * tau;
          if (!act) w = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) x[k][e] -= w * v[e];
        }
    }
    if (tid == 0) flops += 2ull * (h - j) + 4ull * (unsigned long long)(h - j) * (r - j - 1);
  }
#pragma unroll
  for (int k = 0; k < CPG; ++k)
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const int c = 64 * k + g, i = sl + 16 * e;
      if (c < r && i < h && i <= c) out[i + (size_t)c * ldo] = x[k][e];
    }
  if (tid == 0) count_work(K_QR, flops, 0);
}

// Tree step of the TSQR for two stacked triangles: R_a (r x r, upper) over R_b (rb x r, upper
// trapezoidal, rb <= r), factored without touching the zeros.  Step j's reflector has the support
// {row j of R_a} U {rows 0..min(j, rb - 1) of R_b}: it is formed from R_a(j, j) and the top of
// column j of R_b, and changes row j of R_a and those rows of R_b right of column j (2(j + 2)(r - j)
// multiply-adds instead of 2(2r - j)(r - j) for the dense stack).  R_a sits in LDS as a packed upper
// triangle (row j from j (2r - j + 1) / 2, columns j .. r - 1); R_b in registers, column c in the
// 16-lane group c % 64 (slot c / 64), rows sl + 16 e in lane sl.  One barrier per step.  The result
// (the new R_a) replaces slot a; columns near underflow are rescaled as in householder_regs.
template <typename T, int EM, int CPG>
static __device__ void householder_tri_pair(const T* A, const T* B, int ld, T* out, int r, int rb, T* dyn) {
  T* Ra = dyn;                                   // packed upper triangle, r (r + 1) / 2 entries
  T(*vbuf)[16 * EM] = reinterpret_cast<T(*)[16 * EM]>(dyn + (size_t)r * (r + 1) / 2);
  T* sbuf = dyn + (size_t)r * (r + 1) / 2 + 2 * 16 * EM;  // [2]: v0, tau per parity
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6), sub = lane >> 4, sl = lane & 15;
  const int g = tid >> 4;
  auto off = [r](int j) { return j * (2 * r - j + 1) / 2; };
  for (int idx = tid; idx < r * r; idx += QR_THREADS) {
    const int i = idx % r, c = idx / r;
    if (i <= c) Ra[off(i) + (c - i)] = A[i + (size_t)c * ld];
  }
  T x[CPG][EM];
#pragma unroll
  for (int k = 0; k < CPG; ++k)
#pragma unroll
    for (int e = 0; e < EM; ++e) {
      const int c = 64 * k + g, i = sl + 16 * e;
      x[k][e] = (c < r && i < rb && i <= c) ? B[i + (size_t)c * ld] : (T)0;
    }
  __syncthreads();
  unsigned long long flops = 0;
  for (int j = 0; j < r; ++j) {
    const int b = j & 1, go = j & 63, kj = j >> 6;
    const int jb = j < rb - 1 ? j : rb - 1;  // last row of R_b in the reflector's support
    if (wave == (go >> 2)) {
      const bool owner = sub == (go & 3);
#pragma unroll
      for (int k = 0; k < CPG; ++k)
        if (k == kj) {  // wave-uniform
          const T x0 = Ra[off(j)];
          T s = 0, am = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const T v = (sl + 16 * e <= jb) ? x[k][e] : (T)0;
            s += v * v;
            am = fmax(am, fabs(v));
          }
          s = row_sum(s);
          am = fmax(row_max(am), fabs(x0));
          const bool scaled = s < Prec<T>::scale_below && am > (T)0;
          T sc1 = 1, sc2 = 1, unscale = 1;
          if (scaled) {
            constexpr int M = Prec<T>::max_shift;
            const int ex = ilogb(am);
            sc1 = ldexp((T)1, -ex > M ? M : -ex);
            sc2 = ldexp((T)1, -ex > M ? -ex - M : 0);
            unscale = ldexp((T)1, ex);
          }
          T vv[EM];
          T ss = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const T v = (sl + 16 * e <= jb) ? x[k][e] : (T)0;
            vv[e] = scaled ? (v * sc1) * sc2 : v;
            ss += vv[e] * vv[e];
          }
          T x0s = x0;
          if (scaled) {
            x0s = (x0 * sc1) * sc2;
            s = row_sum(ss);
          }
          T tau = 0, v0 = 0, rjj = x0;
          if (s != (T)0) {
            const T nrm = sqrt(x0s * x0s + s);
            const T beta = x0s >= 0 ? -nrm : nrm;
            v0 = x0s - beta;
            tau = (T)1 / (nrm * (nrm + fabs(x0s)));
            rjj = beta * unscale;
          }
          if (owner) {
#pragma unroll
            for (int e = 0; e < EM; ++e) {
              vbuf[b][sl + 16 * e] = vv[e];
              if (tau != (T)0 && sl + 16 * e <= jb) x[k][e] = 0;  // annihilated
            }
            if (sl == 0) {
              sbuf[2 * b] = v0;
              sbuf[2 * b + 1] = tau;
              Ra[off(j)] = rjj;
            }
          }
        }
    }
    __syncthreads();
    const T v0 = sbuf[2 * b], tau = sbuf[2 * b + 1];
    if (tau != (T)0 && 64 * (CPG - 1) + 4 * wave + 3 > j) {
      T v[EM];
#pragma unroll
      for (int e = 0; e < EM; ++e) v[e] = vbuf[b][sl + 16 * e];
#pragma unroll
      for (int k = 0; k < CPG; ++k)
        if (64 * k + 4 * wave + 3 > j && 64 * k + 4 * wave < r) {  // wave-uniform
          const int c = 64 * k + g;
          const bool act = c > j && c < r;
          const T a0 = act ? Ra[off(j) + (c - j)] : (T)0;
          T w = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) w += v[e] * x[k][e];
          w = (row_sum(w) + v0 * a0) * tau;
          if (!act) w = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) x[k][e] -= w * v[e];
          if (act && sl == 0) Ra[off(j) + (c - j)] = a0 - w * v0;
        }
    }
    if (tid == 0) flops += 2ull * (jb + 2) + 4ull * (unsigned long long)(jb + 2) * (r - j - 1);
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += QR_THREADS) {
    const int i = idx % r, c = idx / r;
    out[i + (size_t)c * ld] = i <= c ? Ra[off(i) + (c - i)] : (T)0;
  }
  if (tid == 0) count_work(K_QR, flops, 0);
}

template <typename T>
static __device__ void householder_rows(T* X, int ld, int h, int r) {
  __shared__ T cn[QR_RMAX];  // squared norm of column c below row j, for the next pivot
  __shared__ T red[QR_WAVES];
  __shared__ T sh_v0, sh_tau;
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int jend = (h - 1 < r) ? h - 1 : r;
  if (jend <= 0) return;
  if (wave == 0) {
    T s = 0;
    for (int i = 1 + lane; i < h; i += 64) s += X[i] * X[i];
    s = wave_sum(s);
    if (lane == 0) cn[0] = s;
  }
  __syncthreads();
  unsigned long long flops = 0;
  for (int j = 0; j < jend; ++j) {
    // cn[j] is final for this step (updates below write cn[c] for c > j only), so the branch is
    // uniform over the block; X(j, j) is read by thread 0 alone on the fast path.
    T s = cn[j], x0 = 0, unscale = 1;
    if (s < Prec<T>::scale_below) {
      // Tiny column (off-diagonal factors decay exponentially, so entries near the underflow
      // threshold occur): its squared norm lost precision and 1/(nrm (nrm + |x0|)) could overflow.
      // Rescale rows j.. of the column by a power of two (exact) and recompute the norm; the
      // reflector is unchanged by the scaling, only the diagonal of R is scaled back.
      T am = 0;
      for (int i = j + tid; i < h; i += QR_THREADS) am = fmax(am, fabs(X[i + (size_t)j * ld]));
      am = block_reduce<true>(am, red);
      s = 0;
      x0 = 0;
      if (am > 0) {
        // 2^-e can exceed the largest value when am is subnormal: apply it as two factors
        constexpr int M = Prec<T>::max_shift;
        const int e = ilogb(am);
        const T sc1 = ldexp((T)1, -e > M ? M : -e), sc2 = ldexp((T)1, -e > M ? -e - M : 0);
        unscale = ldexp((T)1, e);
        T ss = 0;
        for (int i = j + tid; i < h; i += QR_THREADS) {
          const T x = (X[i + (size_t)j * ld] * sc1) * sc2;
          X[i + (size_t)j * ld] = x;
          if (i > j) ss += x * x;
        }
        s = block_reduce<false>(ss, red);  // its barriers also publish the scaled column
        if (tid == 0) x0 = X[j + (size_t)j * ld];
      }
    } else if (tid == 0) {
      x0 = X[j + (size_t)j * ld];
    }
    if (tid == 0) {
      if (s == 0) {
        sh_tau = 0;
        sh_v0 = 0;
        X[j + (size_t)j * ld] = x0 * unscale;
      } else {
        const T nrm = sqrt(x0 * x0 + s);
        const T beta = x0 >= 0 ? -nrm : nrm;
        sh_v0 = x0 - beta;
        sh_tau = (T)1 / (nrm * (nrm + fabs(x0)));
        X[j + (size_t)j * ld] = beta * unscale;
      }
    }
    __syncthreads();
    const T tau = sh_tau, v0 = sh_v0;
    const T* vj = X + (size_t)j * ld;  // reflector: v0 at row j, X[i, j] below
    // four trailing columns per wave; the norm below row j+1 of each updated column is recorded
    for (int c0 = j + 1 + 4 * wave; c0 < r; c0 += 4 * QR_WAVES) {
      const int nc = r - c0 < 4 ? r - c0 : 4;
      T* col[4];
      T w[4] = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) col[q] = X + (size_t)(q < nc ? c0 + q : c0) * ld;
      if (tau != 0) {
        for (int i = j + 1 + lane; i < h; i += 64) {
          const T vi = vj[i];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] += vi * col[q][i];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (wave_sum(w[q]) + v0 * col[q][j]) * tau;
      }
      T nn[4] = {0, 0, 0, 0};
      for (int i = j + 1 + lane; i < h; i += 64) {
        const T vi = vj[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T x = col[q][i] - w[q] * vi;
          if (q < nc && tau != 0) col[q][i] = x;
          if (i > j + 1) nn[q] += x * x;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) nn[q] = wave_sum(nn[q]);
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nc) {
            if (tau != 0) col[q][j] -= w[q] * v0;
            cn[c0 + q] = nn[q];
          }
      }
    }
    if (tid == 0) flops += 2ull * (h - j) + 4ull * (unsigned long long)(h - j) * (r - j - 1);
    __syncthreads();
  }
  if (tid == 0) count_work(K_QR, flops, 0);
}

// Blocked Householder (compact WY) for panels held in global memory: NB columns at a time are
// staged in LDS and factored there; the block reflector H_1..H_nb = I - V T V^T (T upper
// triangular) then updates every trailing column with one read and one write of it
// (w = V^T a, y = T^T w, a -= V y), instead of one pass per column.
constexpr int QR_NB = 8;

template <typename T>
static __device__ void householder_rows_blocked(T* X, int ld, int h, int r, T* Vl) {
  // block width: 6 columns in FP64, 8 in FP32 (the most that stay in 128 registers)
  constexpr int NB = std::is_same<T, double>::value ? 6 : QR_NB;
  __shared__ T Tm[QR_NB * QR_NB];  // Tm[q * QR_NB + a] = T(a, q)
  __shared__ T v0s[QR_NB], taus[QR_NB];
  __shared__ T gram[QR_NB * QR_NB];
  __shared__ T red[QR_WAVES];
  __shared__ T sh_v0, sh_tau, sh_beta;
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int jend = (h - 1 < r) ? h - 1 : r;
  unsigned long long flops = 0;
  for (int j0 = 0; j0 < jend; j0 += NB) {
    const int nb = jend - j0 < NB ? jend - j0 : NB;
    const int hp = h - j0;  // panel rows j0..h-1
    // (a) stage the panel columns j0..j0+nb-1, rows j0.. into LDS, row-major: (i, c) at i * NB + c
    for (int idx = tid; idx < hp * nb; idx += QR_THREADS) {
      const int c = idx / hp, i = idx - c * hp;
      Vl[(size_t)i * NB + c] = X[(j0 + i) + (size_t)(j0 + c) * ld];
    }
    __syncthreads();
    // (b) unblocked Householder on the LDS panel
    for (int jj = 0; jj < nb; ++jj) {
      T* vj = Vl + jj;  // column jj, stride NB
      T s = 0;
      for (int i = jj + 1 + tid; i < hp; i += QR_THREADS) s += vj[i * NB] * vj[i * NB];
      s = block_reduce<false>(s, red);
      T unscale = 1;
      if (s < Prec<T>::scale_below) {  // tiny column: exact power-of-two rescaling first (see householder_rows)
        T am = 0;
        for (int i = jj + tid; i < hp; i += QR_THREADS) am = fmax(am, fabs(vj[i * NB]));
        am = block_reduce<true>(am, red);
        s = 0;
        if (am > 0) {
          constexpr int M = Prec<T>::max_shift;
          const int e = ilogb(am);
          const T sc1 = ldexp((T)1, -e > M ? M : -e), sc2 = ldexp((T)1, -e > M ? -e - M : 0);
          unscale = ldexp((T)1, e);
          T ss = 0;
          for (int i = jj + tid; i < hp; i += QR_THREADS) {
            const T x = (vj[i * NB] * sc1) * sc2;
            vj[i * NB] = x;
            if (i > jj) ss += x * x;
          }
          s = block_reduce<false>(ss, red);
        }
      }
      if (tid == 0) {
        const T x0 = vj[jj * NB];
        if (s == 0) {
          sh_tau = 0;
          sh_v0 = 0;
          sh_beta = x0 * unscale;
        } else {
          const T nrm = sqrt(x0 * x0 + s);
          const T beta = x0 >= 0 ? -nrm : nrm;
          sh_v0 = x0 - beta;
          sh_tau = (T)1 / (nrm * (nrm + fabs(x0)));
          sh_beta = beta * unscale;
        }
      }
      __syncthreads();
      const T tau = sh_tau, v0 = sh_v0;
      // columns jj+1..nb-1 of the panel, one per wave
      for (int c = jj + 1 + wave; c < nb; c += QR_WAVES) {
        if (tau == 0) break;
        T* col = Vl + c;
        T w = lane == 0 ? v0 * col[jj * NB] : (T)0;
        for (int i = jj + 1 + lane; i < hp; i += 64) w += vj[i * NB] * col[i * NB];
        w = wave_sum(w) * tau;
        if (lane == 0) col[jj * NB] -= w * v0;
        for (int i = jj + 1 + lane; i < hp; i += 64) col[i * NB] -= w * vj[i * NB];
      }
      __syncthreads();
      // No barrier after these stores: the next column's steps touch other entries until their
      // first reduction's barrier, and sh_* are rewritten only after that.
      if (tid == 0) {
        v0s[jj] = sh_v0;
        taus[jj] = sh_tau;
        vj[jj * NB] = sh_beta;  // R's diagonal; the reflector head lives in v0s
      }
    }
    __syncthreads();
    // (c) Gram of the reflectors (unit structure: v_q = [0..0, v0s[q], V(q+1.., q)])
    for (int pq = wave; pq < nb * nb; pq += QR_WAVES) {
      const int a = pq / nb, q = pq - a * nb;
      if (a >= q) continue;  // T needs v_a^T v_q for a < q
      // rows > q: both are stored; row q: v_a(q) * v0s[q]
      T g = lane == 0 ? Vl[q * NB + a] * v0s[q] : (T)0;
      for (int i = q + 1 + lane; i < hp; i += 64) g += Vl[i * NB + a] * Vl[i * NB + q];
      g = wave_sum(g);
      if (lane == 0) gram[q * QR_NB + a] = g;
    }
    __syncthreads();
    if (tid == 0) {  // T(q, q) = tau_q; T(0:q, q) = -tau_q T(0:q, 0:q) (V_{0:q}^T v_q)
      for (int q = 0; q < nb; ++q) {
        Tm[q * QR_NB + q] = taus[q];
        for (int a = 0; a < q; ++a) {
          T acc = 0;
          for (int c = a; c < q; ++c) acc += Tm[c * QR_NB + a] * gram[q * QR_NB + c];
          Tm[q * QR_NB + a] = -taus[q] * acc;
        }
      }
    }
    // (d) panel back to global: R rows and the reflector entries below them
    for (int idx = tid; idx < hp * nb; idx += QR_THREADS) {
      const int c = idx / hp, i = idx - c * hp;
      X[(j0 + i) + (size_t)(j0 + c) * ld] = Vl[(size_t)i * NB + c];
    }
    __syncthreads();
    // (e) trailing columns: a <- (I - V T V^T)^T a = a - V (T^T (V^T a)), one column per wave
    for (int c = j0 + nb + wave; c < r; c += QR_WAVES) {
      T* col = X + (size_t)c * ld + j0;  // rows j0..h-1
      // rows below nb hold full reflector columns; the first nb rows the unit-triangular head
      T w[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) w[q] = 0;
      if (lane < nb) {
        const T x = col[lane];
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < nb) w[q] += (lane > q ? Vl[lane * NB + q] : (lane == q ? v0s[q] : (T)0)) * x;
      }
      for (int i = nb + lane; i < hp; i += 64) {
        const T x = col[i];
        const T* vr = Vl + (size_t)i * NB;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < nb) w[q] += vr[q] * x;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) w[q] = wave_sum(w[q]);
#pragma unroll
      for (int q = NB - 1; q >= 0; --q) {  // w <- T^T w in place (T upper triangular: y_q uses w_0..w_q)
        T acc = 0;
#pragma unroll
        for (int a = 0; a <= q; ++a) acc += Tm[q * QR_NB + a] * w[a];
        w[q] = q < nb ? acc : (T)0;
      }
      if (lane < nb) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < nb) acc += (lane > q ? Vl[lane * NB + q] : (lane == q ? v0s[q] : (T)0)) * w[q];
        col[lane] -= acc;
      }
      for (int i = nb + lane; i < hp; i += 64) {
        const T* vr = Vl + (size_t)i * NB;
        T acc = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < nb) acc += vr[q] * w[q];
        col[i] -= acc;
      }
    }
    if (tid == 0)
      for (int jj = 0; jj < nb; ++jj)
        flops += 2ull * (hp - jj) + 4ull * (unsigned long long)(hp - jj) * (r - j0 - jj - 1);
    __syncthreads();
  }
  if (tid == 0) count_work(K_QR, flops, 0);
}

// rows covered by slot a after stage s, capped at r
static __device__ __forceinline__ int slot_live_rows(int a, int s, int h0, int rows, int r) {
  long long end = (long long)(a + (1 << s)) * h0;
  if (end > rows) end = rows;
  long long cov = end - (long long)a * h0;
  if (cov < 0) cov = 0;
  return cov < r ? (int)cov : r;
}

// One TSQR stage for one workgroup's tile or pair of slots; false when the workgroup has nothing to
// do at this stage.  The workspace slots hold T values (the FP64-sized buffer is reinterpreted).
template <typename T>
static __device__ __forceinline__ bool qr_stage_body(const QrTask& Tk, const int r, int stage, int* flag,
                                                     T* qlds) {
  constexpr int kLds = QR_LDS_BYTES / (int)sizeof(T);
  const int tid = threadIdx.x;
  T* const work = reinterpret_cast<T*>(Tk.work);
  T* slot;
  int h, ra = 0;
  int ld0, rows0;
  const double* srcM = nullptr;  // stage 0: the FP64 stack
  const T* src0 = nullptr;       // stage s: slot a
  const T* src1 = nullptr;
  int rb = 0;
  if (stage == 0) {
    const int t = blockIdx.x;
    if (t >= Tk.ntiles) return false;
    const int r0 = t * Tk.h0;
    h = Tk.rows - r0;
    if (h > Tk.h0) h = Tk.h0;
    slot = work + (size_t)t * Tk.hs * Tk.rcap;
    srcM = Tk.M + r0;
    ld0 = Tk.ldm;
    rows0 = h;
  } else {
    const int half = 1 << (stage - 1);
    const int a = blockIdx.x << stage, b = a + half;
    if (b >= Tk.ntiles) return false;
    ra = slot_live_rows(a, stage - 1, Tk.h0, Tk.rows, r);
    rb = slot_live_rows(b, stage - 1, Tk.h0, Tk.rows, r);
    slot = work + (size_t)a * Tk.hs * Tk.rcap;
    src0 = slot;
    ld0 = Tk.hs;
    rows0 = ra;
    src1 = work + (size_t)b * Tk.hs * Tk.rcap;
    h = ra + rb;
  }
  // FP64: a stack with no more rows than columns is its own triangular factor up to an orthogonal
  // one (M = I M): the recompression only needs R with M = Q R, so the tile is passed on as it is.
  // (FP32 keeps the Householder factor, whose norm-preserving rounding its error bound assumes.)
  if (std::is_same<T, double>::value && stage == 0 && Tk.ntiles == 1 && h <= r) {
    bool bad = false;
    for (int idx = tid; idx < h * r; idx += QR_THREADS) {
      const int i = idx % h, c = idx / h;
      const double v = srcM[i + (size_t)c * ld0];
      bad |= !(fabs(v) <= DBL_MAX);
      slot[i + (size_t)c * Tk.hs] = (T)v;
    }
    if (bad) atomicOr(flag + Tk.fidx, 16);
    return true;
  }
  // small row tiles: the whole tile in registers
  if (stage == 0 && h <= 128 && r <= 256) {
    householder_regs<T, 8, 4>(srcM, ld0, slot, Tk.hs, h, r, flag, Tk.fidx, qlds);
    return true;
  }
  if (stage == 0 && h <= 256 && r <= 128) {
    householder_regs<T, 16, 2>(srcM, ld0, slot, Tk.hs, h, r, flag, Tk.fidx, qlds);
    return true;
  }
  // two stacked triangles (the first one full): structured combine, R_b in registers
  if (stage > 0 && ra == r && rb >= 1 && r <= 192 && (size_t)r * (r + 1) / 2 + 2 * 16 * 12 + 4 <= (size_t)kLds) {
    const int cpg = (r + 63) / 64, em = (rb + 15) / 16;
    if (cpg == 1) {
      if (em <= 4) householder_tri_pair<T, 4, 1>(src0, src1, Tk.hs, slot, r, rb, qlds);
      else householder_tri_pair<T, 8, 1>(src0, src1, Tk.hs, slot, r, rb, qlds);   // rb <= r <= 64 < 128
    } else if (cpg == 2) {
      if (em <= 4) householder_tri_pair<T, 4, 2>(src0, src1, Tk.hs, slot, r, rb, qlds);
      else householder_tri_pair<T, 8, 2>(src0, src1, Tk.hs, slot, r, rb, qlds);
    } else {
      if (em <= 4) householder_tri_pair<T, 4, 3>(src0, src1, Tk.hs, slot, r, rb, qlds);
      else if (em <= 8) householder_tri_pair<T, 8, 3>(src0, src1, Tk.hs, slot, r, rb, qlds);
      else householder_tri_pair<T, 12, 3>(src0, src1, Tk.hs, slot, r, rb, qlds);
    }
    return true;
  }
  const bool inl = h * r <= kLds;
  T* X = inl ? qlds : slot;
  const int ldx = inl ? h : Tk.hs;
  // gather the panel (stage 0: a row tile of M; stage s: triangle of slot a over triangle of slot b)
  if (stage == 0) {
    bool bad = false;  // non-finite stacked input is reported (value 16)
    for (int idx = tid; idx < rows0 * r; idx += QR_THREADS) {
      const int i = idx % rows0, c = idx / rows0;
      const double v = srcM[i + (size_t)c * ld0];
      bad |= !(fabs(v) <= DBL_MAX);
      X[i + (size_t)c * ldx] = (T)v;
    }
    if (bad) atomicOr(flag + Tk.fidx, 16);
  } else if (inl) {
    for (int idx = tid; idx < rows0 * r; idx += QR_THREADS) {
      const int i = idx % rows0, c = idx / rows0;
      X[i + (size_t)c * ldx] = (i <= c) ? src0[i + (size_t)c * ld0] : (T)0;
    }
  } else {  // in place: clear the reflector entries left below the triangle of slot a
    for (int idx = tid; idx < rows0 * r; idx += QR_THREADS) {
      const int i = idx % rows0, c = idx / rows0;
      if (i > c) X[i + (size_t)c * ldx] = 0;
    }
  }
  if (stage > 0)
    for (int idx = tid; idx < rb * r; idx += QR_THREADS) {
      const int i = idx % rb, c = idx / rb;
      X[(ra + i) + (size_t)c * ldx] = (i <= c) ? src1[i + (size_t)c * Tk.hs] : (T)0;
    }
  __syncthreads();
  if (inl || (size_t)h * QR_NB > (size_t)kLds)
    householder_rows<T>(X, ldx, h, r);
  else
    householder_rows_blocked<T>(X, ldx, h, r, qlds);  // panel in global memory, LDS holds the block reflector
  if (inl) {  // the triangle goes back to the slot
    const int rr = h < r ? h : r;
    for (int idx = tid; idx < rr * r; idx += QR_THREADS) {
      const int i = idx % rr, c = idx / rr;
      slot[i + (size_t)c * Tk.hs] = X[i + (size_t)c * ldx];
    }
  }
  return true;
}

// The triangle of slot 0 (the whole tile when a single FP64 tile has no more rows than columns:
// the stack is its own factor) as the r x r factor R, zero below and beyond; non-finite entries
// are reported (value 32).
template <typename T>
static __device__ __forceinline__ void qr_write_r(const QrTask& Tk, const int r, int* flag, int nthreads) {
  const int rr = Tk.rows < r ? Tk.rows : r;
  const T* work = reinterpret_cast<const T*>(Tk.work);
  bool bad = false;
  const bool full = std::is_same<T, double>::value && Tk.ntiles == 1 && Tk.rows <= r;
  for (int idx = threadIdx.x; idx < r * r; idx += nthreads) {
    const int i = idx % r, c = idx / r;
    const double v = (i < rr && (full || i <= c)) ? (double)work[i + (size_t)c * Tk.hs] : 0.0;
    bad |= !(fabs(v) <= DBL_MAX);
    Tk.R[i + (size_t)c * Tk.ldr] = v;
  }
  if (bad) atomicOr(flag + Tk.fidx, 32);  // the triangular factor came out non-finite
}

// One TSQR stage; the workgroup that completes a task's last stage also writes its R.
template <typename T>
__global__ __launch_bounds__(QR_THREADS) void k_qr_stage(const QrTask* __restrict__ tasks, int stage, int* flag) {
  extern __shared__ __align__(16) unsigned char qlds_raw[];
  T* qlds = reinterpret_cast<T*>(qlds_raw);
  const QrTask Tk = tasks[blockIdx.y];
  const int r = live(Tk.rp, Tk.rcap);
  if (r <= 0) return;
  if (!qr_stage_body<T>(Tk, r, stage, flag, qlds)) return;
  int last = 0;  // a task of ntiles tiles ends at stage ceil(log2 ntiles), in the pair of slot 0
  while ((1 << last) < Tk.ntiles) ++last;
  if (stage == last && blockIdx.x == 0) {
    __syncthreads();
    qr_write_r<T>(Tk, r, flag, QR_THREADS);
  }
}

void launch_qr_stage(const QrTask* d_tasks, int ntasks, int stage, int max_pairs, int* flag, bool fp32,
                     hipStream_t s) {
  if (ntasks <= 0 || max_pairs <= 0) return;
  static std::once_flag lds_ok;
  std::call_once(lds_ok, [] {
    check_lds((const void*)k_qr_stage<double>, QR_LDS_BYTES, "k_qr_stage<double>");
    check_lds((const void*)k_qr_stage<float>, QR_LDS_BYTES, "k_qr_stage<float>");
  });
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    const int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    if (fp32)
      HQ_TIMED(K_QR, s, hipLaunchKernelGGL(k_qr_stage<float>, dim3(max_pairs, nt), dim3(QR_THREADS), QR_LDS_BYTES, s,
                                           d_tasks + t0, stage, flag));
    else
      HQ_TIMED(K_QR, s, hipLaunchKernelGGL(k_qr_stage<double>, dim3(max_pairs, nt), dim3(QR_THREADS), QR_LDS_BYTES, s,
                                           d_tasks + t0, stage, flag));
  }
}

// ----------------------------------------------------------------------------------------------
// Core SVD: pivoted Householder QR (rank-revealing, early stop) + one-sided Jacobi on R_t^T.
// One workgroup per core; a column is worked on by a group of 16 lanes.  For r <= 256 a group keeps
// the rows sl + 16 e of its columns in registers, so all loads of a column are in flight at once,
// and each phase is instantiated for where its operands live (LDS or global memory), so that LDS
// operands are reached with LDS instructions.  Larger cores take looped variants.
// ----------------------------------------------------------------------------------------------
constexpr int SVD_THREADS = 1024;
constexpr int SVD_WAVES = SVD_THREADS / 64;
constexpr int SVD_RMAX = 1024;         // largest core handled
// dynamic LDS: B, C and J when they fit, then the per-core index and norm arrays sized for the
// variant's largest core (160 KiB minus the few static reduction slots)
constexpr int SVD_DYN_BYTES = 163328;

template <typename T>
struct ArgMax { T v; int i; };

template <typename T>
static __device__ __forceinline__ ArgMax<T> wave_argmax(ArgMax<T> a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T v = __shfl_xor(a.v, o, 64);
    const int i = __shfl_xor(a.i, o, 64);
    if (v > a.v || (v == a.v && i < a.i)) { a.v = v; a.i = i; }
  }
  return a;
}

// Register segments of padded columns: a group of G lanes (16 or 32) holds a column, element e
// (e0 <= e < e1, wave-uniform bounds) of lane sl being row sl + G e; elements outside [e0, e1) are
// zero and skipped.  Columns are stored with a leading dimension that is a multiple of G and zero
// rows below their length, so whole elements are always in bounds.
template <int EM, int G, typename T, typename X>
static __device__ __forceinline__ void seg_load(X (&x)[EM], const T* p, int e0, int e1, int sl) {
  const T* q = p + sl;
#pragma unroll
  for (int e = 0; e < EM; ++e) x[e] = (e >= e0 && e < e1) ? (X)q[G * e] : (X)0;
}
template <int EM, int G, typename T, typename X>
static __device__ __forceinline__ void seg_store(const X (&x)[EM], T* p, int e0, int e1, int sl) {
  T* q = p + sl;
#pragma unroll
  for (int e = 0; e < EM; ++e)
    if (e >= e0 && e < e1) q[G * e] = (T)x[e];
}

// Sum over a group of G lanes (one or two DPP rows), returned to every lane of the group.
template <int G, typename T>
static __device__ __forceinline__ T group_sum(T v) {
  v = row_sum(v);
  if constexpr (G == 32) v += __shfl_xor(v, 16, 64);
  return v;
}

// Tangent, cosine and sine of the plane rotation that makes two columns with squared norms a, b
// and inner product g orthogonal: the root of smaller magnitude of t^2 g + t (b - a) - g = 0,
// t = sign(d) h / (|d| + sqrt(d^2 + h^2)) with d = b - a, h = 2 g (sign(0) = +1).  d and h are
// first scaled by one power of two, so their squares neither overflow nor underflow.
template <typename T>
static __device__ __forceinline__ void jacobi_angle(T a, T b, T g, T& tt, T& cs, T& sn) {
  T d = b - a, h = (T)2 * g;
  const int ex = ilogb(fmax(fabs(d), fabs(h)));
  d = ldexp(d, -ex);
  h = ldexp(h, -ex);
  tt = (d >= (T)0 ? h : -h) / (fabs(d) + sqrt(d * d + h * h));
  cs = rsqrt((T)1 + tt * tt);
  sn = cs * tt;
}

// Shared state of one core decomposition.
template <typename T>
struct SvdShared {
  T* cn;          // trailing squared column norms; later sigma^2
  T* vl;          // register path: reflector factors (tau, heads); looped path: current reflector
  int* perm;      // column order of the pivoted QR
  int* ordr;      // singular values in decreasing order
  T* redv;
  ArgMax<T>* reda;
  int* rotated;
  unsigned long long* pairs;
  unsigned long long* rots;
};

// Phase 1: Householder QR with column pivoting of the r x r core Bm, stopped once the trailing
// Frobenius norm is at most qr_thresh (FP32: at least a tenth of B's FP32 noise).  Returns t;
// the reflectors sit below the diagonal of Bm's first t columns with their heads in vhead[] and
// factors in tau[]; perm holds the column order.  Non-finite norms set bit 3 of the status word.
template <typename T, int EM, int G>
static __device__ __forceinline__ int svd_qrcp(T* Bm, const int ldb, const int r, const SvdTask& Tk, int* flag,
                                               const SvdShared<T>& S, T* tau, T* vhead) {
  constexpr bool dbl = std::is_same<T, double>::value;
  constexpr int GPW = 64 / G;  // groups per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6), sub = lane / G, sl = lane & (G - 1);
  T* cn = S.cn;
  int* perm = S.perm;
  for (int c = wave; c < r; c += SVD_WAVES) {
    T s = 0;
    for (int i = lane; i < r; i += 64) s += Bm[i + (size_t)c * ldb] * Bm[i + (size_t)c * ldb];
    s = wave_sum(s);
    if (lane == 0) { cn[c] = s; perm[c] = c; }
  }
  __syncthreads();
  T qth2 = (T)(Tk.qr_thresh * Tk.qr_thresh);
  for (int j = 0; j < r; ++j) {
    // trailing norms and the pivot: one column per thread (r <= SVD_THREADS), and only the waves
    // that hold trailing columns take part (waves issue nothing for the others)
    const int nact = (r - j + 63) >> 6;
    if (wave < nact) {
      T s = 0;
      ArgMax<T> am{(T)-1, 0x7fffffff};
      const int c = j + tid;
      if (c < r) {
        s = cn[c];
        am.v = s;
        am.i = c;
      }
      s = wave_sum(s);
      am = wave_argmax(am);
      if (lane == 0) { S.redv[wave] = s; S.reda[wave] = am; }
    }
    __syncthreads();
    T tot = 0;
    ArgMax<T> best = S.reda[0];
    for (int w = 0; w < nact; ++w) {
      tot += S.redv[w];
      const ArgMax<T> x = S.reda[w];
      if (x.v > best.v || (x.v == best.v && x.i < best.i)) best = x;
    }
    // FP32: stop where the trailing norm reaches a tenth of the FP32 noise level of B
    if (!dbl && j == 0) qth2 = fmax(qth2, (T)0.01 * (T)Tk.fp32_floor * (T)Tk.fp32_floor * tot);
    // every thread reduced the same partials: the decisions are uniform
    const int stop = uniform(tot <= qth2 ? 1 : (!(tot <= Prec<T>::big) || best.i < j || best.i >= r) ? 2 : 0);
    if (stop == 1) return j;
    if (stop == 2) {
      // non-finite trailing norms: no valid pivot exists; report and stop (the caller discards the result)
      if (tid == 0) atomicOr(flag + Tk.fidx, 8);
      return j;
    }
    const int p = uniform(best.i);
    if (p != j) {
      for (int i = tid; i < r; i += SVD_THREADS) {
        const T x = Bm[i + (size_t)j * ldb];
        Bm[i + (size_t)j * ldb] = Bm[i + (size_t)p * ldb];
        Bm[i + (size_t)p * ldb] = x;
      }
      if (tid == 0) {
        const T x = cn[j]; cn[j] = cn[p]; cn[p] = x;
        const int q = perm[j]; perm[j] = perm[p]; perm[p] = q;
      }
      __syncthreads();
    }
    // reflector from the trailing norm of the pivot column (rows j..r-1); computed by the waves with
    // trailing columns and by wave 0, which stores it
    T beta = 0, vj = 0, tj = 0;
    if (wave == 0 || j + 1 + GPW * wave < r) {
      const T nrm = sqrt(cn[j]), x0 = Bm[j + (size_t)j * ldb];
      beta = x0 >= 0 ? -nrm : nrm;
      vj = x0 - beta;
      tj = nrm > 0 ? (T)1 / (nrm * (nrm + fabs(x0))) : (T)0;
    }
    // trailing columns: four per wave, one per group of 16 lanes; uniform control flow around the
    // row reductions, rows of invalid groups predicated off
    if constexpr (EM > 0) {
      if (j + 1 + GPW * wave < r) {
      // whole elements from the one holding row j: the reflector is zero above row j, so rows above
      // j pass through unchanged (and are stored back as they were)
      const int e0 = j / G, e1 = (r + G - 1) / G, jl = j % G;  // row j is lane jl of element e0
      T v[EM];
      seg_load<EM, G>(v, Bm + (size_t)j * ldb, e0, e1, sl);
#pragma unroll
      for (int e = 0; e < EM; ++e)
        if (e == e0) v[e] = sl > jl ? v[e] : (sl == jl ? vj : (T)0);
      for (int cc = j + 1 + GPW * wave; cc < r; cc += GPW * SVD_WAVES) {
        const int c = cc + sub;
        const bool valid = c < r;
        T* col = Bm + (size_t)(valid ? c : cc) * ldb;
        T x[EM];
        seg_load<EM, G>(x, col, e0, e1, sl);
        T w = 0;
#pragma unroll
        for (int e = 0; e < EM; ++e) w += v[e] * x[e];
        w = group_sum<G>(w) * tj;
        T nn = 0;
#pragma unroll
        for (int e = 0; e < EM; ++e) {
          x[e] -= w * v[e];
          if (e != e0 || sl > jl) nn += x[e] * x[e];  // rows below j
        }
        nn = group_sum<G>(nn);
        if (valid) {
          seg_store<EM, G>(x, col, e0, e1, sl);
          if (sl == 0) cn[c] = nn;  // exact trailing norm for the next step
        }
      }
      }
    } else {
      T* vl = S.vl;
      for (int i = j + 1 + tid; i < r; i += SVD_THREADS) vl[i] = Bm[i + (size_t)j * ldb];
      __syncthreads();
      for (int cc = j + 1 + 4 * wave; cc < r; cc += 4 * SVD_WAVES) {
        const int c = cc + sub;
        const bool valid = c < r;
        T* col = Bm + (size_t)(valid ? c : cc) * ldb;
        T w = (sl == 0) ? vj * col[j] : (T)0;
        for (int i = j + 1 + sl; i < r; i += 16) w += vl[i] * col[i];
        w = row_sum(w) * tj;
        if (valid && sl == 0) col[j] -= w * vj;
        T nn = 0;
        for (int i = j + 1 + sl; i < r; i += 16) {
          const T x = col[i] - w * vl[i];
          if (valid) col[i] = x;
          nn += x * x;
        }
        nn = row_sum(nn);
        if (valid && sl == 0) cn[c] = nn;
      }
    }
    __syncthreads();
    if (tid == 0) {
      Bm[j + (size_t)j * ldb] = beta;
      tau[j] = tj;
      vhead[j] = vj;
    }
  }
  return r;
}

// Phases 2-4 for given homes of B (reflectors), C = R_t^T (r x t) and J (t x t):
//   2. one-sided Jacobi on C with rotations accumulated in J, squared column norms tracked through
//      the rotations and recomputed at the start of every sweep;
//   3. singular values (column norms of C J), decreasing order, truncation at thresh (FP32: also at
//      fp32_floor sigma_1), capped at kcap (overflow sets bit 0 of the status word);
//   4. B ~ Q_t J S (Pi W S^{-1})^T with W = C J:
//        Jk[perm[c], o] = W[c, ord(o)] / sigma      (right singular vectors)
//        Wk = Q_t [J[:, ord(o)] / sigma ; 0]         (left singular vectors over sigma)
// Returns the number of sweeps.
// PAD: the columns of C and J have EM G rows of storage each (ldc = ldj = EM G), zero beyond r and t,
// so the rotation loop moves whole register segments with no per-element bounds.
template <typename T, int EM, int G, bool PAD = false>
static __device__ __forceinline__ int svd_tail(const T* Bm, const int ldb, T* C, const int ldc, T* J, const int ldj,
                                               const int r, const int t, const SvdTask& Tk, int* flag,
                                               const SvdShared<T>& S, const T* tau, const T* vhead,
                                               unsigned& my_pairs, unsigned& my_rots, unsigned long long& c2) {
  constexpr bool dbl = std::is_same<T, double>::value;
  constexpr int GPW = 64 / G;  // groups per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6), sub = lane / G, sl = lane & (G - 1);
  // rows padded to multiples of G with zeros (rotations keep them zero)
  const int rpad = (r + G - 1) / G * G, tpad = (t + G - 1) / G * G, er = rpad / G, et = tpad / G;
  const int crows = PAD ? EM * G : rpad, jrows = PAD ? EM * G : tpad;  // rows initialised
  const int ser = PAD ? EM : er, set = PAD ? EM : et;                  // elements moved by the rotations
  for (int idx = tid; idx < crows * t; idx += SVD_THREADS) {
    const int c = idx % crows, i = idx / crows;  // C[c, i] = R[i, c]
    C[c + (size_t)i * ldc] = (c >= i && c < r) ? Bm[i + (size_t)c * ldb] : (T)0;
  }
  // J is read only to form the left singular vectors: without them (Wk null) it is neither set up nor
  // rotated, and C, hence every output, is the same either way
  const bool needJ = Tk.Wk != nullptr;
  if (needJ)
    for (int idx = tid; idx < jrows * t; idx += SVD_THREADS) {
      const int i = idx % jrows, c = idx / jrows;
      J[i + (size_t)c * ldj] = (i == c) ? (T)1 : (T)0;
    }
  __syncthreads();
  // ---- phase 2
  const int tp = t + (t & 1);
  const T tol = (T)4 * Prec<T>::eps * sqrt((T)r);
  T* nrm2 = S.cn;
  int nsweeps = 0;
  for (int sweep = 0; sweep < 40 && t > 1; ++sweep) {
    for (int c = wave; c < t; c += SVD_WAVES) {
      T s = 0;
      for (int i = lane; i < r; i += 64) s += C[i + (size_t)c * ldc] * C[i + (size_t)c * ldc];
      s = wave_sum(s);
      if (lane == 0) nrm2[c] = s;
    }
    if (tid == 0) *S.rotated = 0;
    __syncthreads();
    // Each pair of a round (round-robin order) gets a group of G lanes, 64 / G pairs per wave: dot
    // products reduce inside the group, and up to (64 / G) SVD_WAVES pairs rotate at once.  A group
    // without a valid pair, or whose pair needs no rotation, is predicated off.
    for (int round = 0; round < tp - 1; ++round) {
      for (int pi0 = wave * GPW; pi0 < tp / 2; pi0 += GPW * SVD_WAVES) {
        const int pi = pi0 + sub;
        const int x = pi, y = tp - 1 - pi;
        int px = x - 1 + round, qy = y - 1 + round;  // (x - 1 + round) mod (tp - 1), both < 2 (tp - 1)
        if (px >= tp - 1) px -= tp - 1;
        if (qy >= tp - 1) qy -= tp - 1;
        int pp = (x == 0) ? 0 : 1 + px, qq = (y == 0) ? 0 : 1 + qy;
        if (pp > qq) { const int w0 = pp; pp = qq; qq = w0; }
        const bool valid = pi < tp / 2 && qq < t;
        if (!valid) { pp = 0; qq = 0; }  // harmless addresses for predicated-off groups
        T* cp = C + (size_t)pp * ldc;
        T* cq = C + (size_t)qq * ldc;
        const T a = nrm2[pp], b = nrm2[qq];
        if constexpr (EM > 0) {
          T up[EM], uq[EM];
          seg_load<EM, G>(up, cp, 0, ser, sl);
          seg_load<EM, G>(uq, cq, 0, ser, sl);
          T gg = 0;
#pragma unroll
          for (int e = 0; e < EM; ++e) gg += up[e] * uq[e];
          gg = group_sum<G>(gg);
          // rotate when |g| > tol sqrt(a b), tested without square roots
          const bool rot = valid && a > Prec<T>::tiny && b > Prec<T>::tiny && gg * gg > tol * tol * a * b;
          my_pairs += valid && sl == 0;
          my_rots += rot && sl == 0;
          T tt = 0, cs = 1, sn = 0;
          if (rot) jacobi_angle(a, b, gg, tt, cs, sn);
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const T u2 = cs * up[e] - sn * uq[e], w2 = sn * up[e] + cs * uq[e];
            up[e] = u2;
            uq[e] = w2;
          }
          T ea = a - tt * gg, eb = b + tt * gg;  // exact-arithmetic norms after the rotation
          const bool exact = rot && (!(ea > (T)0.25 * a) || !(eb > (T)0.25 * b));  // cancellation: computed norms
          if (__any(exact)) {  // wave-uniform; rare
            T na = 0, nb = 0;
#pragma unroll
            for (int e = 0; e < EM; ++e) {
              na += up[e] * up[e];
              nb += uq[e] * uq[e];
            }
            na = group_sum<G>(na);
            nb = group_sum<G>(nb);
            if (exact) {
              ea = na;
              eb = nb;
            }
          }
          if (rot) {
            seg_store<EM, G>(up, cp, 0, ser, sl);
            seg_store<EM, G>(uq, cq, 0, ser, sl);
            if (needJ) {
              T* jp = J + (size_t)pp * ldj;
              T* jq = J + (size_t)qq * ldj;
              T vp[EM], vq[EM];
              seg_load<EM, G>(vp, jp, 0, set, sl);
              seg_load<EM, G>(vq, jq, 0, set, sl);
#pragma unroll
              for (int e = 0; e < EM; ++e) {
                const T u2 = cs * vp[e] - sn * vq[e], w2 = sn * vp[e] + cs * vq[e];
                vp[e] = u2;
                vq[e] = w2;
              }
              seg_store<EM, G>(vp, jp, 0, set, sl);
              seg_store<EM, G>(vq, jq, 0, set, sl);
            }
            if (sl == 0) {
              nrm2[pp] = ea;
              nrm2[qq] = eb;
              *S.rotated = 1;
            }
          }
        } else {
          T gg = 0;
          if (valid)
            for (int i = sl; i < r; i += 16) gg += cp[i] * cq[i];
          gg = row_sum(gg);
          const bool rot = valid && a > Prec<T>::tiny && b > Prec<T>::tiny && gg * gg > tol * tol * a * b;
          my_pairs += valid && sl == 0;
          my_rots += rot && sl == 0;
          T tt = 0, cs = 1, sn = 0;
          if (rot) jacobi_angle(a, b, gg, tt, cs, sn);
          T na = 0, nb = 0;
          if (rot)
            for (int i = sl; i < r; i += 16) {
              const T uu = cp[i], w = cq[i];
              const T u2 = cs * uu - sn * w, w2 = sn * uu + cs * w;
              cp[i] = u2;
              cq[i] = w2;
              na += u2 * u2;
              nb += w2 * w2;
            }
          T ea = a - tt * gg, eb = b + tt * gg;
          const bool exact = rot && (!(ea > (T)0.25 * a) || !(eb > (T)0.25 * b));
          if (__any(exact)) {
            na = row_sum(na);
            nb = row_sum(nb);
            if (exact) {
              ea = na;
              eb = nb;
            }
          }
          if (rot) {
            if (needJ) {
              T* jp = J + (size_t)pp * ldj;
              T* jq = J + (size_t)qq * ldj;
              for (int i = sl; i < t; i += 16) {
                const T uu = jp[i], w = jq[i];
                jp[i] = cs * uu - sn * w;
                jq[i] = sn * uu + cs * w;
              }
            }
            if (sl == 0) {
              nrm2[pp] = ea;
              nrm2[qq] = eb;
              *S.rotated = 1;
            }
          }
        }
      }
      __syncthreads();
    }
    ++nsweeps;
    if (!uniform(*S.rotated)) break;
    __syncthreads();
  }
  c2 = wall_clock64();
  // ---- phase 3
  T* sig2 = S.cn;
  int* ordr = S.ordr;
  for (int c = wave; c < t; c += SVD_WAVES) {
    T s = 0;
    for (int i = lane; i < r; i += 64) s += C[i + (size_t)c * ldc] * C[i + (size_t)c * ldc];
    s = wave_sum(s);
    if (!(s <= Prec<T>::big)) {  // NaN or Inf: flagged, and ranked last so that the ordering stays a permutation
      if (lane == 0) atomicOr(flag + Tk.fidx, 8);
      s = 0.0;
    }
    if (lane == 0) sig2[c] = s;
  }
  __syncthreads();
  for (int i = tid; i < t; i += SVD_THREADS) {
    int pos = 0;
    const T si = sig2[i];
    for (int j = 0; j < t; ++j) pos += (sig2[j] > si) || (sig2[j] == si && j < i);
    ordr[pos] = i;
  }
  __syncthreads();
  T th2 = (T)(Tk.thresh * Tk.thresh);
  if (!dbl) {  // FP32: keep sigma > max(thresh, floor * sigma_1)
    T smax = 0;
    for (int i = 0; i < t; ++i) smax = fmax(smax, sig2[i]);
    th2 = fmax(th2, (T)Tk.fp32_floor * (T)Tk.fp32_floor * smax);
  }
  int kk = 0;
  for (int i = 0; i < t; ++i) kk += sig2[i] > th2;
  kk = uniform(kk);
  if (kk > Tk.kcap) {
    if (tid == 0) atomicOr(flag + Tk.fidx, 1);
    kk = Tk.kcap;
  }
  if (tid == 0) *Tk.kout = kk;
  if (Tk.sig)
    for (int i = tid; i < t; i += SVD_THREADS) Tk.sig[i] = sqrt((double)sig2[ordr[i]]);
  // ---- phase 4
  const int* perm = S.perm;
  for (int idx = tid; idx < r * kk; idx += SVD_THREADS) {
    const int c = idx % r, o = idx / r, src = ordr[o];
    const double is = 1.0 / sqrt((double)sig2[src]);
    Tk.Jk[perm[c] + (size_t)o * Tk.ld] = C[c + (size_t)src * ldc] * is;
    if constexpr (EM == 0)
      if (Tk.Wk) Tk.Wk[c + (size_t)o * Tk.ld] = (c < t) ? J[c + (size_t)src * ldj] * is : 0.0;
  }
  if (!Tk.Wk) return nsweeps;  // right singular vectors only (symmetric compressions): no reflector replay
  if constexpr (EM > 0) {
    // Each output column stays in registers of one group through the t reflectors (applied last to
    // first).
    for (int o0 = GPW * wave; o0 < kk; o0 += GPW * SVD_WAVES) {
      const int o = o0 + sub;
      const bool valid = o < kk;
      const int src = ordr[valid ? o : o0];
      const double is = 1.0 / sqrt((double)sig2[src]);
      double x[EM];
      seg_load<EM, G>(x, J + (size_t)src * ldj, 0, et, sl);
#pragma unroll
      for (int e = 0; e < EM; ++e) x[e] *= is;
      for (int j = t - 1; j >= 0; --j) {
        T v[EM];
        const double tj = tau[j], vj = vhead[j];
        if (uniform(tj != 0.0)) {
          const int e0 = j / G, jl = j % G;  // row j is lane jl of element e0
          seg_load<EM, G>(v, Bm + (size_t)j * ldb, e0, er, sl);
#pragma unroll
          for (int e = 0; e < EM; ++e)
            if (e == e0) v[e] = sl > jl ? v[e] : (sl == jl ? (T)vj : (T)0);
          double w = 0.0;
#pragma unroll
          for (int e = 0; e < EM; ++e) w += (double)v[e] * x[e];
          w = group_sum<G>(w) * tj;
#pragma unroll
          for (int e = 0; e < EM; ++e) x[e] -= w * (double)v[e];
        }
      }
      if (valid) seg_store<EM, G>(x, Tk.Wk + (size_t)o * Tk.ld, 0, er, sl);
    }
  } else {
    __syncthreads();
    for (int j = t - 1; j >= 0; --j) {
      const double tj = tau[j], vj = vhead[j];
      if (uniform(tj != 0.0)) {  // the output columns, one per group of 16 lanes
        const T* vcol = Bm + (size_t)j * ldb;
        for (int o0 = 4 * wave; o0 < kk; o0 += 4 * SVD_WAVES) {
          const int o = o0 + sub;
          const bool valid = o < kk;
          double* col = Tk.Wk + (size_t)(valid ? o : o0) * Tk.ld;
          double w = (sl == 0) ? vj * col[j] : 0.0;
          for (int i = j + 1 + sl; i < r; i += 16) w += vcol[i] * col[i];
          w = row_sum(w) * tj;
          if (valid) {
            if (sl == 0) col[j] -= w * vj;
            for (int i = j + 1 + sl; i < r; i += 16) col[i] -= w * vcol[i];
          }
        }
      }
      __syncthreads();
    }
  }
  return nsweeps;
}

// T = double: FP64 throughout.  T = float: the core is rounded to FP32, everything runs in FP32, and
// truncation uses max(thresh, fp32_floor sigma_1) (singular values below that are FP32 noise); the
// outputs stay FP64.  Workspace buffers (C, Jw, aux) are reinterpreted as T.
template <typename T, int EM, int G>
static __device__ __forceinline__ void svd_run(const SvdTask& Tk, int* flag, const int r, unsigned char* raw,
                                               const SvdShared<T>& S0) {
  constexpr bool dbl = std::is_same<T, double>::value;
  // largest core of the variant; its arrays (norms, reflector factors or the current reflector,
  // pivot order, singular value order) sit after the data region
  constexpr int RM = EM > 0 ? EM * G : SVD_RMAX;
  constexpr int ARR = RM * (int)sizeof(T) * (EM > 0 ? 3 : 2) + 2 * RM * (int)sizeof(int);
  constexpr int SVD_LDS = ((SVD_DYN_BYTES - ARR) / (int)sizeof(T)) & ~1;
  static_assert(SVD_LDS >= 16384, "data region below 16384 entries");
  T* const slds = reinterpret_cast<T*>(raw);
  T* const cn = slds + SVD_LDS;
  T* const vl = cn + RM;
  int* const perm = reinterpret_cast<int*>(vl + (EM > 0 ? 2 * RM : RM));
  const SvdShared<T> S{cn, vl, perm, perm + RM, S0.redv, S0.reda, S0.rotated, S0.pairs, S0.rots};
  const int tid = threadIdx.x;
  // reflector factors: in LDS on the register path (t <= r <= RM: tau in [0, RM), heads in [RM, 2 RM)), else in the aux workspace
  T* tau = EM > 0 ? S.vl : reinterpret_cast<T*>(Tk.aux);
  T* vhead = EM > 0 ? S.vl + RM : reinterpret_cast<T*>(Tk.aux) + r;
  // global copy of B in T: the input buffer itself (FP64), or the upper half of the C workspace
  T* const Bglob = dbl ? reinterpret_cast<T*>(Tk.B) : reinterpret_cast<T*>(Tk.C) + (size_t)Tk.ld * Tk.ld;
  const unsigned long long c0 = wall_clock64();
  unsigned long long c1 = c0, c2 = c0;
  unsigned my_pairs = 0, my_rots = 0;  // per group lane 0, summed once at the end
  // ---- phase 1 on B with rows padded by zeros to rpad (a multiple of G, at most Tk.ld)
  const int rpad = (r + G - 1) / G * G;
  const bool bl = rpad * r <= SVD_LDS;
  int t;
  if (bl) {
    for (int idx = tid; idx < rpad * r; idx += SVD_THREADS) {
      const int i = idx % rpad, c = idx / rpad;
      slds[idx] = i < r ? (T)Tk.B[i + (size_t)c * Tk.ld] : (T)0;
    }
    __syncthreads();
    t = svd_qrcp<T, EM, G>(slds, rpad, r, Tk, flag, S, tau, vhead);
  } else {
    for (int idx = tid; idx < rpad * r; idx += SVD_THREADS) {
      const int i = idx % rpad, c = idx / rpad;
      const size_t o = i + (size_t)c * Tk.ld;
      if (i >= r) Bglob[o] = (T)0;
      else if (!dbl) Bglob[o] = (T)Tk.B[o];
    }
    __syncthreads();
    t = svd_qrcp<T, EM, G>(Bglob, Tk.ld, r, Tk, flag, S, tau, vhead);
  }
  __syncthreads();
  c1 = wall_clock64();
  if (t == 0) {
    if (tid == 0) *Tk.kout = 0;
    return;
  }
  // ---- phases 2-4: C = R_t^T (rpad x t) and J (tpad x t) in LDS when they fit (B stays there too
  // if there is room)
  const int tpad = (t + G - 1) / G * G;
  const int nB = rpad * r, nC = rpad * t, nJ = tpad * t;
  int nsweeps;
  if (EM > 0 && 2 * EM * G * t <= SVD_LDS && !(bl && nB + nC + nJ <= SVD_LDS && EM * G > 2 * rpad)) {
    // C and J in LDS with whole-segment columns; B (reflectors) in global memory
    if (bl) {
      for (int idx = tid; idx < nB; idx += SVD_THREADS) Bglob[(idx % rpad) + (size_t)(idx / rpad) * Tk.ld] = slds[idx];
      __syncthreads();
    }
    constexpr int LD = EM > 0 ? EM * G : 1;
    nsweeps = svd_tail<T, EM, G, true>(Bglob, Tk.ld, slds, LD, slds + LD * t, LD, r, t, Tk, flag, S, tau, vhead,
                                       my_pairs, my_rots, c2);
  } else if (bl && nB + nC + nJ <= SVD_LDS) {
    nsweeps = svd_tail<T, EM, G>(slds, rpad, slds + nB, rpad, slds + nB + nC, tpad, r, t, Tk, flag, S, tau, vhead,
                              my_pairs, my_rots, c2);
  } else {
    if (bl) {  // free the LDS: reflectors (and the zero padding) back to global
      for (int idx = tid; idx < nB; idx += SVD_THREADS) Bglob[(idx % rpad) + (size_t)(idx / rpad) * Tk.ld] = slds[idx];
      __syncthreads();
    }
    T* const Cg = reinterpret_cast<T*>(Tk.C);
    T* const Jg = reinterpret_cast<T*>(Tk.Jw);
    constexpr int LD = EM > 0 ? EM * G : 1;
    if (nC + nJ <= SVD_LDS)
      nsweeps = svd_tail<T, EM, G>(Bglob, Tk.ld, slds, rpad, slds + nC, tpad, r, t, Tk, flag, S, tau, vhead, my_pairs,
                                my_rots, c2);
    else if (EM > 0 && LD * t <= SVD_LDS && Tk.ld >= LD)  // C in LDS with whole-segment columns, J global
      nsweeps = svd_tail<T, EM, G, true>(Bglob, Tk.ld, slds, LD, Jg, Tk.ld, r, t, Tk, flag, S, tau, vhead, my_pairs,
                                         my_rots, c2);
    else if (nC <= SVD_LDS)  // C (the longer columns) in LDS, J global
      nsweeps = svd_tail<T, EM, G>(Bglob, Tk.ld, slds, rpad, Jg, Tk.ld, r, t, Tk, flag, S, tau, vhead, my_pairs,
                                my_rots, c2);
    else if (nJ <= SVD_LDS)
      nsweeps = svd_tail<T, EM, G>(Bglob, Tk.ld, Cg, Tk.ld, slds, tpad, r, t, Tk, flag, S, tau, vhead, my_pairs,
                                my_rots, c2);
    else
      nsweeps = svd_tail<T, EM, G>(Bglob, Tk.ld, Cg, Tk.ld, Jg, Tk.ld, r, t, Tk, flag, S, tau, vhead, my_pairs,
                                my_rots, c2);
  }
  if ((threadIdx.x & (G - 1)) == 0 && my_pairs) {  // counted on the first lane of each group
    atomicAdd(S.pairs, (unsigned long long)my_pairs);
    atomicAdd(S.rots, (unsigned long long)my_rots);
  }
  __syncthreads();
  if (tid == 0) {
    const int kk = *Tk.kout;
    unsigned long long f = 0;
    for (int j = 0; j < t; ++j)
      f += 2ull * (r - j) + 6ull * (unsigned long long)(r - j) * (r - j - 1) + 4ull * (r - j) * kk;
    f += *S.pairs * 6ull * r + *S.rots * (6ull * r + (Tk.Wk ? 6ull * t : 0ull)) + 2ull * r * t;
    count_work(K_SVD, f, 0);
    if (g_prof_on) {
      const unsigned long long c3 = wall_clock64();
      atomicAdd(&g_svdstat[0], c1 - c0);
      atomicAdd(&g_svdstat[1], c2 - c1);
      atomicAdd(&g_svdstat[2], c3 - c2);
      atomicAdd(&g_svdstat[3], (unsigned long long)r);
      atomicAdd(&g_svdstat[4], (unsigned long long)t);
      atomicAdd(&g_svdstat[5], (unsigned long long)nsweeps);
      atomicAdd(&g_svdstat[6], 1ull);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(SVD_THREADS) void k_svd(const SvdTask* __restrict__ tasks, int* flag) {
  extern __shared__ __align__(16) unsigned char svd_raw[];
  const SvdTask Tk = tasks[blockIdx.x];
  int rfull = uniform(*Tk.rp);
  if (rfull <= Tk.keep_below) {  // kept as it is: Jk = I (r columns)
    const int k = rfull < Tk.kcap ? rfull : Tk.kcap;
    if (rfull > Tk.kcap && threadIdx.x == 0) atomicOr(flag + Tk.fidx, 1);
    for (int idx = threadIdx.x; idx < Tk.ld * k; idx += SVD_THREADS) {
      const int i = idx % Tk.ld, c = idx / Tk.ld;
      Tk.Jk[i + (size_t)c * Tk.ld] = i == c ? 1.0 : 0.0;
    }
    if (threadIdx.x == 0) *Tk.kout = k < 0 ? 0 : k;
    return;
  }
  if (rfull > SVD_RMAX) rfull = SVD_RMAX;
  const int r = rfull < Tk.rlim ? rfull : Tk.rlim;
  if (r <= 0) {
    if (threadIdx.x == 0) *Tk.kout = 0;
    return;
  }
  if (Tk.ld < ((r + 15) & ~15)) {  // workspaces must hold the rows padded to a multiple of 16 (32 above 256)
    if (threadIdx.x == 0) {
      atomicOr(flag + Tk.fidx, 8);
      *Tk.kout = 0;
    }
    return;
  }
  __shared__ T redv[SVD_WAVES];
  __shared__ ArgMax<T> reda[SVD_WAVES];
  __shared__ int rotated;
  __shared__ unsigned long long sh_pairs, sh_rots;
  if (threadIdx.x == 0) { sh_pairs = 0; sh_rots = 0; }
  const SvdShared<T> S{nullptr, nullptr, nullptr, nullptr, redv, reda, &rotated, &sh_pairs, &sh_rots};
  if (r <= 128)
    svd_run<T, 8, 16>(Tk, flag, r, svd_raw, S);
  else if (r <= 256)
    svd_run<T, 16, 16>(Tk, flag, r, svd_raw, S);
  else if (r <= 512 && Tk.ld >= ((r + 31) & ~31))
    svd_run<T, 16, 32>(Tk, flag, r, svd_raw, S);  // 32-lane groups
  else
    svd_run<T, 0, 16>(Tk, flag, r, svd_raw, S);
  if (rfull > r) {  // rows r..rfull-1 of the singular vectors of a core with zero rows and columns there
    __syncthreads();
    const int kk = *Tk.kout, nr = rfull - r;
    for (int idx = threadIdx.x; idx < nr * kk; idx += SVD_THREADS) {
      const size_t o = (size_t)(r + idx % nr) + (size_t)(idx / nr) * Tk.ld;
      Tk.Jk[o] = 0.0;
      if (Tk.Wk) Tk.Wk[o] = 0.0;
    }
  }
}

void launch_svd(const SvdTask* d_tasks, int ntasks, int* flag, bool fp32, hipStream_t s) {
  if (ntasks <= 0) return;
  static std::once_flag lds_ok;
  std::call_once(lds_ok, [] {
    check_lds((const void*)k_svd<double>, SVD_DYN_BYTES, "k_svd<double>");
    check_lds((const void*)k_svd<float>, SVD_DYN_BYTES, "k_svd<float>");
  });
  if (fp32)
    HQ_TIMED(K_SVD, s, hipLaunchKernelGGL(k_svd<float>, dim3(ntasks), dim3(SVD_THREADS), SVD_DYN_BYTES, s, d_tasks,
                                          flag));
  else
    HQ_TIMED(K_SVD, s, hipLaunchKernelGGL(k_svd<double>, dim3(ntasks), dim3(SVD_THREADS), SVD_DYN_BYTES, s, d_tasks,
                                          flag));
}

// ----------------------------------------------------------------------------------------------
// Cholesky of the small SPD matrix M = G + E (one workgroup), C = lower factor, M = C C^T.  The lower
// triangle is kept as 4 x 4 tiles in registers, TPT tiles per thread (order up to SPD_REG), or, above
// that, packed (entry (i, k), i >= k, at i (i + 1) / 2 + k) in the task's workspace.  Register path,
// two columns per step: at step j, column j is final and column j + 1 lacks only column j's
// contribution; both sit in LDS, published by their owners in the step before.  After one barrier
// every thread forms the pivots M(j, j) and M(j + 1, j + 1) - M(j + 1, j)^2 / M(j, j) itself, writes
// its share of columns j and j + 1 of C, applies the rank-two update of both columns to its entries
// right of column j + 1 and, if it owns columns j + 2 and j + 3, publishes them.  One barrier per two
// columns, no pivot search.  Orders whose tiles need two per thread take one column per step (the
// two-column step's temporaries would not stay in registers beside two tiles).  The launch has as many threads as the largest order's tiles need
// (blockDim.x, a multiple of 64), so that small orders wait on few waves at each barrier.
// ----------------------------------------------------------------------------------------------
constexpr int SPD_THREADS = 1024;
static __device__ __forceinline__ int pk(int i, int k) { return i >= k ? i * (i + 1) / 2 + k : k * (k + 1) / 2 + i; }
// (x, y), x >= y, of packed index q = x (x + 1) / 2 + y
static __device__ __forceinline__ void unpack_lower(int q, int& x, int& y) {
  x = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
  if ((x + 1) * (x + 2) / 2 <= q) ++x;
  if (x * (x + 1) / 2 > q) --x;
  y = q - x * (x + 1) / 2;
}
static __device__ __forceinline__ double gram_entry(const SpdCholTask& T, int i, int k, int e0) {
  double v = T.G[i + (size_t)k * T.ldg];
  if (i == k && i >= e0) v += 1.0;
  return v;
}

// 4 x 4 tiles of the lower triangle of an order-r matrix (r <= 4 sqrt(2 SPD_THREADS) covers one tile per thread)
static __host__ __device__ __forceinline__ int spd_tiles(int r) {
  const int nb = (r + 3) / 4;
  return nb * (nb + 1) / 2;
}

template <int TPT>
static __device__ void spd_chol_regs(const SpdCholTask& T, int r, double (*cols)[2][SPD_REG], int* flag,
                                     const int nthr) {
  const int tid = threadIdx.x;
  const int ntile = spd_tiles(r);
  const int e0 = T.ep ? uniform(*T.ep) : r;
  double a[TPT][4][4];
  int bi[TPT], bk[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int q = tid + t * nthr;
    int x = -1, y = -1;
    if (q < ntile) unpack_lower(q, x, y);
    bi[t] = x;
    bk[t] = y;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * x + u, k = 4 * y + v;
        a[t][u][v] = (x >= 0 && i < r && k < r && i >= k) ? gram_entry(T, i, k, e0) : 0.0;
      }
    if (y == 0) {  // publish columns 0 and 1 (tiles of block column 0 hold rows 4x .. 4x + 3 of them)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * x + u < r) {
          cols[0][0][4 * x + u] = a[t][u][0];
          cols[0][1][4 * x + u] = a[t][u][1];
        }
    }
  }
  unsigned long long flops = 0;
  int j = 0;
  for (; j < r; j += 2) {
    lds_barrier();
    const double* c0 = cols[(j >> 1) & 1][0];
    const double* c1 = cols[(j >> 1) & 1][1];
    double* n0 = cols[((j >> 1) + 1) & 1][0];
    double* n1 = cols[((j >> 1) + 1) & 1][1];
    const bool two = j + 1 < r;
    const double d0 = c0[j];
    if (!(d0 > 0.0)) {  // M is positive definite by construction; report a breakdown, stop
      if (tid == 0) atomicOr(flag + T.fidx, 2);
      break;
    }
    const double inv0 = 1.0 / d0, s0 = rsqrt(d0);
    const double g = two ? c0[j + 1] * inv0 : 0.0;  // column j+1 gets -g * column j
    const double d1 = two ? c1[j + 1] - g * c0[j + 1] : 1.0;
    const bool bad1 = two && !(d1 > 0.0);
    const double inv1 = bad1 ? 0.0 : 1.0 / d1, s1 = bad1 ? 0.0 : rsqrt(d1);
    double* Cj = T.C + (size_t)j * T.ldc;
    for (int i = tid; i < r; i += nthr) Cj[i] = i >= j ? c0[i] * s0 : 0.0;
    if (bad1) {  // column j is done; the breakdown is at j + 1
      if (tid == 0) atomicOr(flag + T.fidx, 2);
      j += 1;
      break;
    }
    if (!two) {
      j += 1;
      break;
    }
    double* Cj1 = T.C + (size_t)(j + 1) * T.ldc;
    for (int i = tid; i < r; i += nthr) Cj1[i] = i >= j + 1 ? (c1[i] - g * c0[i]) * s1 : 0.0;
    const int bj = (j + 2) >> 2, cjn = (j + 2) & 3;  // tile column holding columns j + 2, j + 3
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      if (bi[t] < 0 || 4 * bi[t] + 3 <= j + 1) continue;  // rows all at or above j + 1: nothing left to update
      double v0[4], v1[4];  // columns j and j + 1 (the latter after column j's step) at this tile's columns
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 4 * bk[t] + v;
        const bool kin = k > j + 1 && k < r;
        v0[v] = kin ? c0[k] : 0.0;
        v1[v] = kin ? c1[k] - g * v0[v] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = 4 * bi[t] + u;
        const bool iin = i > j + 1 && i < r;
        const double ci0 = iin ? c0[i] : 0.0;
        const double ui0 = ci0 * inv0, ui1 = iin ? (c1[i] - g * ci0) * inv1 : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) a[t][u][v] -= ui0 * v0[v] + ui1 * v1[v];
      }
      if (bk[t] == bj && j + 2 < r) {  // publish columns j + 2 and j + 3 (static indices by comparison)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (v == cjn) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = 4 * bi[t] + u;
              if (i >= j + 2 && i < r) {
                n0[i] = a[t][u][v];
                if (v + 1 < 4) n1[i] = a[t][u][v + 1];
              }
            }
          }
      }
    }
    if (tid == 0) {
      const unsigned long long m0 = (unsigned long long)(r - j), m1 = m0 - 1;
      flops += m0 * m0 + m0 + m1 * m1 + m1;
    }
  }
  if (j > r) j = r;
  if (tid == 0) {
    *T.kout = j;
    count_work(K_POTRF, flops, 8ull * r * (r + j));
  }
}

// Orders whose tiles need two per thread: one column per step (the two-column step's temporaries
// would not stay in registers beside two tiles).
template <int TPT>
static __device__ void spd_chol_regs_1col(const SpdCholTask& T, int r, double (*cols)[2][SPD_REG], int* flag) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nb = (r + 3) / 4, ntile = nb * (nb + 1) / 2;
  const int e0 = T.ep ? uniform(*T.ep) : r;
  double a[TPT][4][4];
  int bi[TPT], bk[TPT];
  double* colp[2] = {cols[0][0], cols[1][0]};
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int q = tid + t * nthr;
    int x = -1, y = -1;
    if (q < ntile) unpack_lower(q, x, y);
    bi[t] = x;
    bk[t] = y;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * x + u, k = 4 * y + v;
        a[t][u][v] = (x >= 0 && i < r && k < r && i >= k) ? gram_entry(T, i, k, e0) : 0.0;
      }
    if (y == 0) {  // publish column 0 (tiles of block column 0 hold rows 4x .. 4x + 3 of it)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * x + u < r) colp[0][4 * x + u] = a[t][u][0];
    }
  }
  unsigned long long flops = 0;
  int j = 0;
  for (; j < r; ++j) {
    lds_barrier();
    const double* cj = colp[j & 1];
    double* cn = colp[(j + 1) & 1];
    const double d = cj[j];
    if (!(d > 0.0)) {  // M is positive definite by construction; report a breakdown, stop
      if (tid == 0) atomicOr(flag + T.fidx, 2);
      break;
    }
    const double inv = 1.0 / d, sinv = 1.0 / sqrt(d);
    double* Cj = T.C + (size_t)j * T.ldc;
    for (int i = tid; i < r; i += nthr) Cj[i] = i >= j ? cj[i] * sinv : 0.0;
    const int bj = (j + 1) >> 2, cjn = (j + 1) & 3;  // tile column holding column j + 1
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      if (bi[t] < 0 || 4 * bi[t] + 3 <= j) continue;  // rows all at or above j: nothing left to update
      double cu[4], cv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = 4 * bi[t] + u, k = 4 * bk[t] + u;
        cu[u] = (i > j && i < r) ? cj[i] * inv : 0.0;
        cv[u] = (k > j && k < r) ? cj[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) a[t][u][v] -= cu[u] * cv[v];
      if (bk[t] == bj && j + 1 < r) {  // publish column j + 1 (selected by comparison: static indices)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (v == cjn) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = 4 * bi[t] + u;
              if (i >= j + 1 && i < r) cn[i] = a[t][u][v];
            }
          }
      }
    }
    if (tid == 0) {
      const unsigned long long m = (unsigned long long)(r - j);
      flops += m * m + m;
    }
  }
  if (tid == 0) {
    *T.kout = j;
    count_work(K_POTRF, flops, 8ull * r * (r + j));
  }
}

// Orders above SPD_REG: the packed triangle in the task's workspace, entries spread flat.
static __device__ void spd_chol_global(const SpdCholTask& T, int r, double* A, int* flag) {
  const int tid = threadIdx.x;
  const int e0 = T.ep ? uniform(*T.ep) : r;
  const int np0 = r * (r + 1) / 2;
  for (int q = tid; q < np0; q += blockDim.x) {
    int i, k;
    unpack_lower(q, i, k);
    A[q] = gram_entry(T, i, k, e0);
  }
  unsigned long long flops = 0;
  int j = 0;
  for (; j < r; ++j) {
    __syncthreads();
    const double d = A[pk(j, j)];
    if (!(d > 0.0)) {
      if (tid == 0) atomicOr(flag + T.fidx, 2);
      break;
    }
    const double inv = 1.0 / d, sinv = 1.0 / sqrt(d);
    double* Cj = T.C + (size_t)j * T.ldc;
    for (int i = tid; i < r; i += blockDim.x) Cj[i] = i >= j ? A[pk(i, j)] * sinv : 0.0;
    // trailing triangle: rows and columns j + 1 .. r - 1, packed relative to j + 1
    const int m = r - j - 1, npair = m * (m + 1) / 2;
    for (int q = tid; q < npair; q += blockDim.x) {
      int x, y;
      unpack_lower(q, x, y);
      const int i = j + 1 + x, k = j + 1 + y;
      A[pk(i, k)] -= A[pk(i, j)] * A[pk(k, j)] * inv;
    }
    if (tid == 0) flops += (unsigned long long)(m + 1) * (m + 1);
  }
  if (tid == 0) {
    *T.kout = j;
    count_work(K_POTRF, flops, 8ull * r * (r + j));
  }
}

// TPT = 1: launches whose largest order's tiles fit one per thread; TPT = 2: launches with a larger
// order (1024 threads; two tiles per thread up to SPD_REG, the packed workspace above), in a kernel
// of their own so that the common one keeps every tile in registers without spilling.  A task whose
// tiles fit one per thread takes the two-column path in either kernel.
template <int TPT>
__global__ __launch_bounds__(SPD_THREADS) void k_spd_chol(const SpdCholTask* __restrict__ tasks, int* flag) {
  __shared__ double cols[2][2][SPD_REG];
  const SpdCholTask T = tasks[blockIdx.x];
  const int r = uniform(*T.rp);
  if (r <= 0) {
    if (threadIdx.x == 0) *T.kout = 0;
    return;
  }
  if (r > T.kcap || r > kMaxStack) {
    if (threadIdx.x == 0) {
      atomicOr(flag + T.fidx, r > kMaxStack ? 4 : 1);
      *T.kout = 0;
    }
    return;
  }
  const int nt = spd_tiles(r), nthr = blockDim.x;
  // the variant depends on the order alone (never on what shares the launch), so that a task's
  // factor is the same bit for bit in any batch
  if (nt <= SPD_THREADS && nt <= nthr) {
    // Waves past this order's tiles leave at once: a wave that has ended is not waited for at the
    // barriers of the others, which then synchronise only the waves that hold tiles.
    const int nact = (nt + 63) / 64 * 64;
    if ((int)threadIdx.x >= nact) return;
    spd_chol_regs<1>(T, r, cols, flag, nact);
  }
  else if (TPT == 2 && r <= SPD_REG && nt <= 2 * nthr)
    spd_chol_regs_1col<2>(T, r, cols, flag);
  else if (T.work)
    spd_chol_global(T, r, T.work, flag);
  else if (threadIdx.x == 0) {  // no workspace for an order above the register path: report
    atomicOr(flag + T.fidx, 8);
    *T.kout = 0;
  }
}

void launch_spd_chol(const SpdCholTask* d_tasks, int ntasks, int max_r, int* flag, hipStream_t s) {
  if (ntasks <= 0) return;
  constexpr size_t dyn = 0;
  // one tile per thread when the largest order allows it, else the full workgroup
  const int need = spd_tiles(max_r < 1 ? 1 : max_r);
  const bool one = need <= SPD_THREADS;
  const int threads = one ? (need + 63) / 64 * 64 : SPD_THREADS;
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    const int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    if (one)
      HQ_TIMED(K_POTRF, s, hipLaunchKernelGGL(k_spd_chol<1>, dim3(nt), dim3(threads), dyn, s, d_tasks + t0, flag));
    else
      HQ_TIMED(K_POTRF, s, hipLaunchKernelGGL(k_spd_chol<2>, dim3(nt), dim3(threads), dyn, s, d_tasks + t0, flag));
  }
}

// ----------------------------------------------------------------------------------------------
// Leaf Cholesky and triangular inverse for m <= 128, with the tile in registers, by 4 x 4 blocks.
// The lower triangle of the tile (padded with the identity to a multiple of 4) is cut into 4 x 4
// blocks, one per thread (at most 528), numbered column by column.  Block step J factors block
// column J and, in the same sweep, eliminates block row J of X = L^{-1} (right-looking on [L | I]):
//   A: every block in a row below J - 1 applies step J - 1: trailing blocks (column >= J) subtract
//      L_{i,J-1} L_{c,J-1}^T; blocks of X subtract L_{i,J-1} X_{J-1,c}, the former panel blocks
//      (column J - 1, which held L_{i,J-1}) starting from zero.  The diagonal block then holds the
//      Schur complement A_JJ; its thread factors it (4 x 4 Cholesky) and inverts the factor,
//      W = L_JJ^{-1}, which is also X_JJ.
//   B: the panel L_{iJ} = A_{iJ} W^T, and block row J of X scaled by W, are published.
// Two barriers per block step; the panel, the row of X and W each need one LDS buffer, since every
// read of one happens in the half step before its next write.
// A (lower part of an SPD tile) is read; B receives L^{-1} (zero above the diagonal).
constexpr int CI_MAX = 128;
constexpr int CI_PAD = CI_MAX + 4;
constexpr int CI_THREADS = 576;  // nine waves cover the 528 blocks of a 128 x 128 tile

// 4 x 4 Cholesky of the lower part of d and the inverse of its factor, in one thread: w = L^{-1}
// (lower).  A pivot that is not positive (or not finite) is replaced by 1 and reported.
static __device__ __forceinline__ void chol4_inv(const double (&d)[4][4], double (&w)[4][4], int valid_rows,
                                                 bool& bad) {
  double l[4][4], rinv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) l[r][c] = r >= c ? d[r][c] : 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double p = l[k][k];
    if (!(p > 0.0)) {
      if (k < valid_rows) bad = true;
      p = 1.0;
    }
    const double rs = rsqrt(p);
    rinv[k] = rs;
    l[k][k] = p * rs;
#pragma unroll
    for (int r = k + 1; r < 4; ++r) l[r][k] *= rs;
#pragma unroll
    for (int c = k + 1; c < 4; ++c)
#pragma unroll
      for (int r = c; r < 4; ++r) l[r][c] -= l[r][k] * l[c][k];
  }
  // forward substitution, column by column of the identity
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r < c) {
        w[r][c] = 0.0;
      } else if (r == c) {
        w[r][c] = rinv[r];
      } else {
        double acc = 0.0;
#pragma unroll
        for (int k = c; k < r; ++k) acc += l[r][k] * w[k][c];
        w[r][c] = -acc * rinv[r];
      }
    }
  }
}

__global__ __launch_bounds__(CI_THREADS) void k_chol_inv(const LeafTask* __restrict__ tasks, int* flag) {
  const LeafTask T = tasks[blockIdx.x];
  const int m = T.m, tid = threadIdx.x;
  const int nb = (m + 3) >> 2;
  const bool own = tid < nb * (nb + 1) / 2;
  int bi = 0, bc = 0;
  if (own) {  // block number tid, column by column: column bc holds blocks bi = bc .. nb - 1
    int t = tid;
    while (t >= nb - bc) {
      t -= nb - bc;
      ++bc;
    }
    bi = bc + t;
  }
  const int r0 = 4 * bi, c0 = 4 * bc;
  double a[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = r0 + r, k = c0 + c;
      double v = 0.0;
      if (own) {
        if (i < m && k < m) {
          if (i >= k) v = T.A[i + (size_t)k * T.lda];
        } else if (i == k) {
          v = 1.0;
        }
      }
      a[r][c] = v;
    }
  __shared__ double pan[4][CI_PAD];   // panel L_{:,J}: column k of the block column, by row
  __shared__ double xrow[4][CI_PAD];  // block row J of X: row k, by column
  __shared__ double wsh[4][4];        // W = L_JJ^{-1}
  bool bad = false;
  for (int J = 0; J < nb; ++J) {
    // ---- A: step J - 1 applied below row block J - 1; the diagonal block factored
    if (own && bi >= J) {
      if (J > 0) {
        const double* ysrc = bc >= J ? &pan[0][0] : &xrow[0][0];  // L_{c,J-1}^T or X_{J-1,c}
        double li[4][4], y[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) li[r][k] = pan[k][r0 + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) y[k][c] = ysrc[k * CI_PAD + c0 + c];
        }
        const bool fresh = bc == J - 1;  // former panel block: X starts from zero
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double acc = fresh ? 0.0 : a[r][c];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc -= li[r][k] * y[k][c];
            a[r][c] = acc;
          }
      }
      if (bi == J && bc == J) {
        double w[4][4];
        chol4_inv(a, w, m - r0, bad);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a[r][c] = w[r][c];
            wsh[r][c] = w[r][c];
          }
      }
    }
    __syncthreads();
    // ---- B: the panel L_{iJ} = A_{iJ} W^T and block row J of X (W X_{Jc}; X_JJ = W) published
    if (own && (bc == J || bi == J)) {
      double w[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) w[r][c] = r >= c ? wsh[r][c] : 0.0;
      if (bc == J && bi > J) {
        double o[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= c; ++k) acc += a[r][k] * w[c][k];
            o[r][c] = acc;
          }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a[r][c] = o[r][c];
            pan[c][r0 + r] = o[r][c];
          }
      } else if (bi == J && bc < J) {
        double o[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= r; ++k) acc += w[r][k] * a[k][c];
            o[r][c] = acc;
          }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a[r][c] = o[r][c];
            xrow[r][c0 + c] = o[r][c];
          }
      } else {  // the diagonal block: X_JJ = W
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) xrow[r][c0 + c] = a[r][c];
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(flag + T.fidx, 2);  // breakdown: a unit pivot kept the rest finite
  // ---- B = L^{-1}: owned blocks, and zeros in the blocks above the diagonal
  if (own)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = r0 + r, k = c0 + c;
        if (i < m && k < m) T.B[i + (size_t)k * T.ldb] = i >= k ? a[r][c] : 0.0;
      }
  for (int idx = tid; idx < m * m; idx += CI_THREADS) {
    const int i = idx % m, k = idx / m;
    if ((i >> 2) < (k >> 2)) T.B[i + (size_t)k * T.ldb] = 0.0;
  }
  if (tid == 0) count_work(K_POTRF, 2ull * m * m * m / 3, 0);
}

void launch_chol_inv(const LeafTask* d_tasks, int ntasks, int max_m, int* flag, hipStream_t s) {
  if (ntasks <= 0) return;
  if (max_m > CI_MAX) throw std::runtime_error("launch_chol_inv: leaf larger than 128");
  HQ_TIMED(K_POTRF, s, hipLaunchKernelGGL(k_chol_inv, dim3(ntasks), dim3(CI_THREADS), 0, s, d_tasks, flag));
}


// ----------------------------------------------------------------------------------------------
// Leaf-level elementwise: out = alpha*X + beta*op(Y) + gamma*I.
// ----------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_leaf_axpy(const LeafAxpy* __restrict__ tasks) {
  const LeafAxpy T = tasks[blockIdx.y];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= T.m * T.m) return;
  const int i = idx % T.m, c = idx / T.m;
  double v = T.gamma * (i == c ? 1.0 : 0.0);
  if (T.alpha != 0.0) v += T.alpha * T.X[i + (size_t)c * T.ldx];
  if (T.beta != 0.0) v += T.beta * (T.transY ? T.Y[c + (size_t)i * T.ldy] : T.Y[i + (size_t)c * T.ldy]);
  T.out[i + (size_t)c * T.ldo] = v;
}
void launch_leaf_axpy(const LeafAxpy* d_tasks, int ntasks, int max_m, hipStream_t s) {
  if (ntasks <= 0) return;
  const int bx = (max_m * max_m + 255) / 256;
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    const int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    HQ_TIMED(K_LEAF, s, hipLaunchKernelGGL(k_leaf_axpy, dim3(bx, nt), dim3(256), 0, s, d_tasks + t0));
  }
}

__global__ void k_fill_int(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_int(int* d, const int* s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}
void launch_fill_int(int* p, int value, int count, hipStream_t s) {
  if (count > 0) {
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, value, count);
    check_launch("fill_int");
  }
}
void launch_copy_int(int* dst, const int* src, int count, hipStream_t s) {
  if (count > 0) {
    hipLaunchKernelGGL(k_copy_int, dim3((count + 255) / 256), dim3(256), 0, s, dst, src, count);
    check_launch("copy_int");
  }
}
__global__ void k_copy_ints(const IntCopy* __restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *list[i].d = *list[i].s;
}
void launch_copy_ints(const IntCopy* d_list, int n, hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(k_copy_ints, dim3((n + 255) / 256), dim3(256), 0, s, d_list, n);
    check_launch("copy_ints");
  }
}

// ----------------------------------------------------------------------------------------------
// Band -> HODLR of X0 = (A - shift I) * inv_scale.  Exact: leaves are the dense band pieces and
// every off-diagonal block is the b x b corner next to the diagonal, stored with rank b.
// ----------------------------------------------------------------------------------------------
static __device__ __forceinline__ double band_at(const BandDesc& bd, int64_t i, int64_t j) {
  int64_t d = i - j;
  if (d < 0) { d = -d; const int64_t t = i; i = j; j = t; }
  if (d > bd.b) return 0.0;
  return bd.ab[d + j * bd.ldab];
}

__global__ __launch_bounds__(256) void k_band_leaves(BandDesc bd, double* leaves, int ldl, const int64_t* lo,
                                                     const int* ms) {
  const int leaf = blockIdx.y, m = ms[leaf];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= m * m) return;
  const int i = idx % m, c = idx / m;
  const int64_t g0 = lo[leaf];
  double v = band_at(bd, g0 + i, g0 + c) * bd.inv_scale;
  if (i == c) v -= bd.shift * bd.inv_scale;
  leaves[(size_t)leaf * ldl * ldl + i + (size_t)c * ldl] = v;
}
void launch_band_leaves(BandDesc bd, double* leaves, int ldl, const int64_t* d_leaf_lo, const int* d_leaf_m,
                        int nleaves, hipStream_t s) {
  hipLaunchKernelGGL(k_band_leaves, dim3((ldl * ldl + 255) / 256, nleaves), dim3(256), 0, s, bd, leaves, ldl,
                     d_leaf_lo, d_leaf_m);
  check_launch("band_leaves");
}

__global__ __launch_bounds__(256) void k_band_blocks(BandDesc bd, const BandBlockTask* __restrict__ tasks) {
  const BandBlockTask T = tasks[blockIdx.y];
  const int b = bd.b, tid = blockIdx.x * 256 + threadIdx.x;
  // lower block rows [mid, mid+rows_b) x cols [mid-rows_a, mid): Ul = [I_b; 0], Vl = corner^T
  if (tid < T.rows_b * b) {
    const int i = tid % T.rows_b, t = tid / T.rows_b;
    const double u = (i == t) ? 1.0 : 0.0;
    T.Ul[i + (size_t)t * T.ldf] = u;
    T.Vu[i + (size_t)t * T.ldf] = u;
  }
  if (tid < T.rows_a * b) {
    const int jj = tid % T.rows_a, t = tid / T.rows_a;
    const int64_t gi = T.mid + t, gj = T.mid - T.rows_a + jj;
    const double v = (gj >= T.mid - b) ? band_at(bd, gi, gj) * bd.inv_scale : 0.0;
    T.Vl[jj + (size_t)t * T.ldf] = v;
    T.Uu[jj + (size_t)t * T.ldf] = v;
  }
  if (tid == 0) {
    *T.rank_l = b;
    *T.rank_u = b;
  }
}
void launch_band_blocks(BandDesc bd, const BandBlockTask* d_tasks, int ntasks, int max_rows, hipStream_t s) {
  if (ntasks <= 0) return;
  const int bx = (max_rows * bd.b + 255) / 256;
  hipLaunchKernelGGL(k_band_blocks, dim3(bx, ntasks), dim3(256), 0, s, bd, d_tasks);
  check_launch("band_blocks");
}

}  // namespace hq

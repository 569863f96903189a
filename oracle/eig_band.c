/*
 * CPU FP64 reference eigen-solver for a symmetric banded matrix -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use this file.  It
 * shares no code with the HIP path.  It computes the quantities that define the spectral
 * projector of the problem statement (Sec. 1 of the paper): the eigenvalues below a shift
 * mu and their eigenvectors, from which Pi = V V^T.
 *
 *   count      : #{lambda_i < sigma} by Sylvester's law of inertia -- the number of negative
 *                pivots of the unpivoted LDL^T factorisation of A - sigma*I (for b = 1 this
 *                is the classical Sturm-sequence recurrence q_i = (d_i - sigma) - e_{i-1}^2/q_{i-1}).
 *   bisection  : lambda_k by interval halving on count(sigma) >= k, started from the
 *                Gershgorin interval.
 *   inverse it.: (A - lambda_k I) x_{t+1} = x_t with a banded LU with partial pivoting,
 *                a deterministic pseudo-random start vector (seed k), three steps.
 *
 * Storage: LAPACK lower band, ab[i + j*ld] = A(j+i, j), 0 <= i <= b.
 * Everything is plain, unblocked, obviously-correct code.  Parallelism (OpenMP) is only
 * across independent eigenvalues.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double aget(const double* ab, long ld, int b, long i, long j) {
  /* A(i,j) of the symmetric band matrix, zero outside the band */
  long d = i - j;
  if (d < 0) { d = -d; long t = i; i = j; j = t; }
  if (d > b) return 0.0;
  return ab[d + j * ld];
}

double oracle_norm_inf(long n, int b, const double* ab, long ld) {
  double m = 0.0;
  for (long i = 0; i < n; ++i) {
    double s = 0.0;
    long j0 = i - b < 0 ? 0 : i - b, j1 = i + b > n - 1 ? n - 1 : i + b;
    for (long j = j0; j <= j1; ++j) s += fabs(aget(ab, ld, b, i, j));
    if (s > m) m = s;
  }
  return m;
}

void oracle_gershgorin(long n, int b, const double* ab, long ld, double* lo, double* hi) {
  double gl = INFINITY, gu = -INFINITY;
  for (long i = 0; i < n; ++i) {
    double r = 0.0;
    long j0 = i - b < 0 ? 0 : i - b, j1 = i + b > n - 1 ? n - 1 : i + b;
    for (long j = j0; j <= j1; ++j)
      if (j != i) r += fabs(aget(ab, ld, b, i, j));
    double a = aget(ab, ld, b, i, i);
    if (a - r < gl) gl = a - r;
    if (a + r > gu) gu = a + r;
  }
  *lo = gl;
  *hi = gu;
}

/* Number of eigenvalues strictly below sigma.  work: n*b doubles + n doubles (may be NULL). */
long oracle_count(long n, int b, const double* ab, long ld, double sigma, double pivmin, double* work) {
  long neg = 0;
  if (b == 1) {
    double q = ab[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++neg;
    for (long i = 1; i < n; ++i) {
      double e = ab[1 + (i - 1) * ld];
      q = (ab[i * ld] - sigma) - e * e / q;
      if (fabs(q) < pivmin) q = -pivmin; /* a zero pivot counts as negative */
      if (q < 0) ++neg;
    }
    return neg;
  }
  double* own = NULL;
  if (!work) own = work = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(b + 1));
  double* L = work;              /* L(i,j) for 1 <= i-j <= b at L[(i-j-1) + j*b] */
  double* d = work + (size_t)n * b;
  for (long j = 0; j < n; ++j) {
    double s = aget(ab, ld, b, j, j) - sigma;
    long k0 = j - b < 0 ? 0 : j - b;
    for (long k = k0; k < j; ++k) {
      double l = L[(j - k - 1) + k * b];
      s -= l * l * d[k];
    }
    if (fabs(s) < pivmin) s = -pivmin;
    d[j] = s;
    if (s < 0) ++neg;
    long i1 = j + b > n - 1 ? n - 1 : j + b;
    for (long i = j + 1; i <= i1; ++i) {
      double t = aget(ab, ld, b, i, j);
      long kk0 = i - b < 0 ? 0 : i - b;
      for (long k = kk0; k < j; ++k) t -= L[(i - k - 1) + k * b] * L[(j - k - 1) + k * b] * d[k];
      L[(i - j - 1) + j * b] = t / s;
    }
  }
  free(own);
  return neg;
}

static double pivmin_of(long n, int b, const double* ab, long ld) {
  double m = 1.0;
  for (long j = 0; j < n; ++j)
    for (int i = 1; i <= b && j + i < n; ++i) {
      double v = ab[i + j * ld];
      if (v * v > m) m = v * v;
    }
  return DBL_MIN * m;
}

/* lambda_k (1-based k) by bisection. */
static double bisect_one(long n, int b, const double* ab, long ld, long k, double gl, double gu, double pivmin,
                         double* work) {
  double lo = gl, hi = gu;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    if (oracle_count(n, b, ab, ld, mid, pivmin, work) >= k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

/* eigenvalues lambda_{k0} .. lambda_{k1} (1-based, inclusive) into lam[0 .. k1-k0] */
void oracle_bisect(long n, int b, const double* ab, long ld, long k0, long k1, double* lam) {
  double gl, gu;
  oracle_gershgorin(n, b, ab, ld, &gl, &gu);
  double w = gu - gl;
  gl -= 2.0 * DBL_EPSILON * fabs(gl) + 1e-300 + 1e-14 * w;
  gu += 2.0 * DBL_EPSILON * fabs(gu) + 1e-300 + 1e-14 * w;
  double pivmin = pivmin_of(n, b, ab, ld);
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(b + 1));
#pragma omp for schedule(dynamic, 4)
    for (long k = k0; k <= k1; ++k) lam[k - k0] = bisect_one(n, b, ab, ld, k, gl, gu, pivmin, work);
    free(work);
  }
}

/* ---- banded LU with partial pivoting (kl = ku = b; U gets bandwidth 2b) ---- */
/* W has ldw = 3b+1 rows; A(i,j) lives at W[(2b + i - j) + j*ldw] (LAPACK gbtrf layout). */
static void gb_factor(long n, int b, double* W, long ldw, long* piv, double tiny) {
  int kl = b, ku = b, kv = ku + kl;
  for (long j = 0; j < n; ++j) {
    long km = (kl < n - 1 - j) ? kl : n - 1 - j;
    /* pivot search in column j, rows j..j+km */
    long p = 0;
    double best = fabs(W[kv + j * ldw]);
    for (long i = 1; i <= km; ++i) {
      double v = fabs(W[kv + i + j * ldw]);
      if (v > best) { best = v; p = i; }
    }
    piv[j] = j + p;
    long ju = j + kv < n - 1 ? j + kv : n - 1; /* last column touched by row swap */
    if (p != 0) {
      for (long c = j; c <= ju; ++c) {
        double* x = &W[kv + j - c + c * ldw];
        double* y = &W[kv + j + p - c + c * ldw];
        double t = *x; *x = *y; *y = t;
      }
    }
    double piv_v = W[kv + j * ldw];
    if (fabs(piv_v) < tiny) { piv_v = (piv_v < 0 ? -tiny : tiny); W[kv + j * ldw] = piv_v; }
    for (long i = 1; i <= km; ++i) W[kv + i + j * ldw] /= piv_v;
    for (long c = j + 1; c <= ju; ++c) {
      double u = W[kv + j - c + c * ldw];
      if (u == 0.0) continue;
      for (long i = 1; i <= km; ++i) W[kv + j + i - c + c * ldw] -= W[kv + i + j * ldw] * u;
    }
  }
}

static void gb_solve(long n, int b, const double* W, long ldw, const long* piv, double* x) {
  int kl = b, kv = 2 * b;
  for (long j = 0; j < n; ++j) { /* L solve with the interchanges */
    long p = piv[j];
    if (p != j) { double t = x[j]; x[j] = x[p]; x[p] = t; }
    long km = (kl < n - 1 - j) ? kl : n - 1 - j;
    for (long i = 1; i <= km; ++i) x[j + i] -= W[kv + i + j * ldw] * x[j];
  }
  for (long j = n - 1; j >= 0; --j) { /* U solve, U(i,j) for j-2b <= i <= j */
    x[j] /= W[kv + j * ldw];
    long i0 = j - kv < 0 ? 0 : j - kv;
    for (long i = i0; i < j; ++i) x[i] -= W[kv + i - j + j * ldw] * x[j];
  }
}

static uint64_t splitmix(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/*
 * Eigenvectors for the eigenvalues lam[0..m-1] (ascending) by inverse iteration, all
 * eigenvalues in parallel.  V is n x m column-major (ldv = n).  Three steps per vector from a
 * deterministic pseudo-random start (splitmix64 stream keyed by seed and k).
 */
void oracle_inverse_iteration(long n, int b, const double* ab, long ld, long m, const double* lam, long seed,
                              double* V) {
  double anorm = oracle_norm_inf(n, b, ab, ld);
  double tiny = DBL_EPSILON * anorm;
  long ldw = 3 * b + 1;
#pragma omp parallel
  {
    double* W = (double*)malloc(sizeof(double) * (size_t)ldw * (size_t)n);
    long* piv = (long*)malloc(sizeof(long) * (size_t)n);
#pragma omp for schedule(dynamic, 8)
    for (long k = 0; k < m; ++k) {
      memset(W, 0, sizeof(double) * (size_t)ldw * (size_t)n);
      for (long j = 0; j < n; ++j) {
        long i0 = j - b < 0 ? 0 : j - b, i1 = j + b > n - 1 ? n - 1 : j + b;
        for (long i = i0; i <= i1; ++i) W[(2 * b + i - j) + j * ldw] = aget(ab, ld, b, i, j) - (i == j ? lam[k] : 0.0);
      }
      gb_factor(n, b, W, ldw, piv, tiny);
      double* x = V + (size_t)k * n;
      uint64_t st = (uint64_t)seed * 0x100000001B3ull + (uint64_t)k;
      for (long i = 0; i < n; ++i) x[i] = ((double)(splitmix(&st) >> 11) * 0x1.0p-53) - 0.5;
      for (int it = 0; it < 3; ++it) {
        gb_solve(n, b, W, ldw, piv, x);
        double nrm = 0.0;
        for (long i = 0; i < n; ++i) nrm += x[i] * x[i];
        nrm = sqrt(nrm);
        for (long i = 0; i < n; ++i) x[i] /= nrm;
      }
    }
    free(W);
    free(piv);
  }
}

/*
 * Windowed modified Gram-Schmidt, in eigenvalue order: v_k loses its components along every
 * earlier v_q with lam[k] - lam[q] <= ortol (two passes), then is normalised.  Only span(V)
 * matters for Pi, and vectors of well separated eigenvalues are already orthogonal to working
 * precision, so the window (LAPACK dstein's cluster radius 1e-3*||A||) is enough.
 */
void oracle_window_mgs(long n, long m, const double* lam, double ortol, double* V) {
  long q0 = 0;
  for (long k = 0; k < m; ++k) {
    while (lam[k] - lam[q0] > ortol) ++q0;
    double* x = V + (size_t)k * n;
    for (int pass = 0; pass < 2; ++pass)
      for (long q = q0; q < k; ++q) {
        const double* y = V + (size_t)q * n;
        double dot = 0.0;
        for (long i = 0; i < n; ++i) dot += y[i] * x[i];
        for (long i = 0; i < n; ++i) x[i] -= dot * y[i];
      }
    double nrm = 0.0;
    for (long i = 0; i < n; ++i) nrm += x[i] * x[i];
    nrm = sqrt(nrm);
    for (long i = 0; i < n; ++i) x[i] /= nrm;
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

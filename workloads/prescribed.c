/* Banded test matrices with a prescribed spectrum (Sec. 6.1 of the paper), in band storage.
 *
 * Starting from diag(lam), for i = n-1, ..., 1 (0-based) a plane rotation of coordinates (i-1, i),
 * chosen from the pair (a_ii, 1), is applied as a similarity; for i <= n-1-b it pushes one entry
 * just outside the band (distance b+1 from the diagonal, in row i-1), which is chased towards the
 * bottom right corner with further rotations, each removing the entry and creating the next one b
 * rows further down.  The working storage keeps b+2 diagonals (the band plus the bulge), so a step
 * costs O(b) and a chase O(n) rotations at most: O(n^2) flops in all instead of the dense O(n^3).
 * Input generation only: it builds A from its eigenvalues and holds none of the method's arithmetic. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double* w;  /* entry (j + d, j), 0 <= d <= b + 1, at w[j * (b + 2) + d] */
  int64_t n;
  int b;
} band_t;

static inline double* at(band_t* A, int64_t i, int64_t j) {
  if (i < j) { int64_t t = i; i = j; j = t; }
  return A->w + j * (A->b + 2) + (i - j);
}
static inline double get(band_t* A, int64_t i, int64_t j) {
  const int64_t d = i > j ? i - j : j - i;
  if (i < 0 || j < 0 || i >= A->n || j >= A->n || d > A->b + 1) return 0.0;
  return *at(A, i, j);
}
static inline void put(band_t* A, int64_t i, int64_t j, double v) {
  const int64_t d = i > j ? i - j : j - i;
  if (i < 0 || j < 0 || i >= A->n || j >= A->n || d > A->b + 1) return;
  *at(A, i, j) = v;
}

static void rot(double f, double g, double* c, double* s) {
  const double r = hypot(f, g);
  if (r == 0.0) { *c = 1.0; *s = 0.0; return; }
  *c = f / r;
  *s = g / r;
}

/* A <- G^T A G for the rotation of coordinates (p, q = p + 1): rows p, q become
 * (c x_p + s x_q, -s x_p + c x_q), and the same for columns. */
static void apply(band_t* A, int64_t p, double c, double s) {
  const int64_t q = p + 1, lo = p - A->b - 1, hi = q + A->b + 1;
  for (int64_t j = lo; j <= hi; ++j) {
    if (j < 0 || j >= A->n || j == p || j == q) continue;
    const double xp = get(A, p, j), xq = get(A, q, j);
    put(A, p, j, c * xp + s * xq);
    put(A, q, j, -s * xp + c * xq);
  }
  const double app = get(A, p, p), aqq = get(A, q, q), apq = get(A, p, q);
  /* [c s; -s c] [app apq; apq aqq] [c -s; s c] */
  const double t0 = c * app + s * apq, t1 = c * apq + s * aqq;
  const double u0 = -s * app + c * apq, u1 = -s * apq + c * aqq;
  put(A, p, p, t0 * c + t1 * s);
  put(A, p, q, -t0 * s + t1 * c);
  put(A, q, q, -u0 * s + u1 * c);
}

/* ab: lower band storage (n x ld, C order: ab[j * ld + d] = A(j + d, j)), ld >= b + 1.
 * Returns 0, or -1 when the workspace cannot be allocated. */
int prescribed_band(int64_t n, int b, const double* lam, double* ab, int64_t ld) {
  band_t A;
  A.n = n;
  A.b = b;
  A.w = (double*)calloc((size_t)n * (size_t)(b + 2), sizeof(double));
  if (!A.w) return -1;
  for (int64_t j = 0; j < n; ++j) A.w[j * (b + 2)] = lam[j];
  double c, s;
  for (int64_t i = n - 1; i >= 1; --i) {
    rot(get(&A, i, i), 1.0, &c, &s);
    apply(&A, i - 1, c, s);
    /* chase the entry outside the band: row r, column r + b + 1 */
    for (int64_t r = i - 1; r + b + 1 < n;) {
      const int64_t cc = r + b + 1;
      const double g = get(&A, r, cc);
      if (g == 0.0) break;
      rot(get(&A, r, cc - 1), g, &c, &s);
      apply(&A, cc - 1, c, s);
      put(&A, r, cc, 0.0);
      r = cc - 1;
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= b; ++d) ab[j * ld + d] = (j + d < n) ? A.w[j * (b + 2) + d] : 0.0;
  free(A.w);
  return 0;
}

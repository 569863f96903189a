/* The oracle's band eigensolver under AddressSanitizer and UndefinedBehaviorSanitizer: Sturm counts,
 * bisection against the closed-form spectrum of the tridiagonal Laplacian, inverse iteration and
 * the windowed re-orthogonalisation, on a tridiagonal and a banded case. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

long oracle_count(long n, int b, const double* ab, long ld, double sigma, double pivmin, double* work);
void oracle_bisect(long n, int b, const double* ab, long ld, long k0, long k1, double* lam);
void oracle_inverse_iteration(long n, int b, const double* ab, long ld, long m, const double* lam, long seed,
                              double* V);
void oracle_window_mgs(long n, long m, const double* lam, double ortol, double* V);

int main(void) {
  int failures = 0;
  const long n = 60;
  double* ab = calloc(2 * n, sizeof(double)); /* tridiag(-1, 2, -1), lower band storage */
  for (long i = 0; i < n; ++i) {
    ab[2 * i] = 2.0;
    if (i + 1 < n) ab[2 * i + 1] = -1.0;
  }
  double* lam = malloc(n * sizeof(double));
  oracle_bisect(n, 1, ab, 2, 1, n, lam);
  for (long k = 1; k <= n; ++k) {
    const double ref = 2.0 - 2.0 * cos(k * 3.14159265358979323846 / (n + 1));
    if (fabs(lam[k - 1] - ref) > 1e-12) {
      printf("FAIL eigenvalue %ld: %.17g vs %.17g\n", k, lam[k - 1], ref);
      ++failures;
    }
  }
  double* work = malloc(3 * n * sizeof(double));
  if (oracle_count(n, 1, ab, 2, 2.0, 1e-300, work) != n / 2) {
    printf("FAIL count\n");
    ++failures;
  }
  const long m = 8;
  double* V = malloc((size_t)n * m * sizeof(double));
  oracle_inverse_iteration(n, 1, ab, 2, m, lam, 3, V);
  oracle_window_mgs(n, m, lam, 1e-3, V);
  for (long j = 0; j < m; ++j) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += V[i + j * n] * V[i + j * n];
    if (fabs(s - 1.0) > 1e-10) {
      printf("FAIL norm %ld\n", j);
      ++failures;
    }
  }
  /* a pentadiagonal band */
  const int b = 2;
  double* ab2 = calloc((size_t)(b + 1) * n, sizeof(double));
  srand(5);
  for (long i = 0; i < n; ++i)
    for (int d = 0; d <= b && i + d < n; ++d) ab2[(b + 1) * i + d] = (double)rand() / RAND_MAX - 0.5;
  double* lam2 = malloc(n * sizeof(double));
  oracle_bisect(n, b, ab2, b + 1, 1, n, lam2);
  for (long k = 1; k < n; ++k)
    if (!(lam2[k] >= lam2[k - 1])) {
      printf("FAIL order %ld\n", k);
      ++failures;
    }
  free(ab); free(lam); free(work); free(V); free(ab2); free(lam2);
  printf(failures ? "failed %d\n" : "ok\n", failures);
  return failures ? 1 : 0;
}

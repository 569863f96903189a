// Zolotarev coefficients for Zolo-pd (see zolo.h).
#include "zolo.h"

#include <cmath>
#include <stdexcept>

namespace hq {
namespace {
constexpr double kPi = 3.14159265358979323846;

// log(sinh(x)) for x > 0 without overflow.
double log_sinh(double x) { return x > 20.0 ? x - std::log(2.0) + std::log1p(-std::exp(-2.0 * x)) : std::log(std::sinh(x)); }
// asinh(exp(L)) without overflow.
double asinh_exp(double L) { return L > 20.0 ? L + std::log(2.0) : std::asinh(std::exp(L)); }
}  // namespace

double ellipk_complement(double l) {
  // K(k) = pi / (2 AGM(1, sqrt(1 - k^2))); for k = l' = sqrt(1 - l^2) that is AGM(1, l).
  double a = 1.0, b = l;
  for (int i = 0; i < 200 && std::fabs(a - b) > 0x1p-60 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return kPi / (2.0 * a);
}

double jacobi_sc_complement(double u, double l) {
  // sc(u | 1 - l^2) = -i sn(iu | l^2).  The arithmetic-geometric mean recurrence for sn(z | l^2)
  // (a_0 = 1, b_0 = sqrt(1 - l^2), c_0 = l; a_{n+1} = (a_n + b_n) / 2, b_{n+1} = sqrt(a_n b_n),
  // c_{n+1} = (a_n - b_n) / 2 = c_n^2 / (4 a_{n+1}); then phi_N = 2^N a_N z and
  // phi_{n-1} = (phi_n + asin(c_n / a_n sin phi_n)) / 2, sn = sin phi_0) at z = iu keeps every phi
  // purely imaginary, phi_n = i psi_n: sin -> i sinh, asin(i y) -> i asinh(y), and sc = sinh(psi_0).
  // With sinh growing like exp(2^n a_n u), the recurrence may stop only once
  // (c_N / a_N) sinh(psi_N) is negligible (not merely c_N), which for u close to K' takes several
  // more steps than for real arguments; log(c_n) is carried so that nothing underflows or overflows.
  double a[64], lc[64];
  double aa = 1.0, bb = std::sqrt((1.0 - l) * (1.0 + l));
  a[0] = aa;
  lc[0] = std::log(l);
  int n = 0;
  while (n < 62 && lc[n] - std::log(a[n]) + std::ldexp(a[n] * u, n) > -50.0) {
    const double an = 0.5 * (aa + bb), bn = std::sqrt(aa * bb);
    aa = an;
    bb = bn;
    ++n;
    a[n] = aa;
    lc[n] = 2.0 * lc[n - 1] - std::log(4.0 * aa);
  }
  double psi = std::ldexp(a[n] * u, n);
  for (int k = n; k >= 1; --k) psi = 0.5 * (psi + asinh_exp(lc[k] - std::log(a[k]) + log_sinh(psi)));
  return std::sinh(psi);
}

ZoloStep zolo_step(double l, int r) {
  if (!(l >= 1e-150 && l < 1.0) || r < 1 || r > 16) throw std::invalid_argument("zolo_step: l or r out of range");
  ZoloStep z;
  z.r = r;
  z.l = l;
  z.c.assign(2 * r + 1, 0.0);
  z.a.assign(r + 1, 0.0);
  const double Kp = ellipk_complement(l);
  for (int i = 1; i <= 2 * r; ++i) {
    const double s = jacobi_sc_complement(i * Kp / (2 * r + 1), l);
    z.c[i] = l * l * s * s;
  }
  // residues of prod_k (x^2 + c_{2k}) / (x^2 + c_{2k-1}) = 1 + sum_j a_j / (x^2 + c_{2j-1}) at
  // x^2 = -c_{2j-1}
  for (int j = 1; j <= r; ++j) {
    double num = 1.0, den = 1.0;
    for (int k = 1; k <= r; ++k) {
      num *= z.c[2 * k] - z.c[2 * j - 1];
      if (k != j) den *= z.c[2 * k - 1] - z.c[2 * j - 1];
    }
    z.a[j] = num / den;
  }
  double m = 1.0, f = l;
  for (int j = 1; j <= r; ++j) {
    m *= (1.0 + z.c[2 * j - 1]) / (1.0 + z.c[2 * j]);
    f *= (l * l + z.c[2 * j]) / (l * l + z.c[2 * j - 1]);
  }
  z.mhat = m;
  z.lnext = std::fmin(m * f, 1.0);
  return z;
}

std::vector<ZoloStep> zolo_schedule(double l0, double delta, int r, int max_steps) {
  // at least one step (X0 is scaled, not yet a sign); success when 1 - l_K <= delta
  auto run = [&](int rr, int cap, bool& ok) {
    std::vector<ZoloStep> v;
    double l = l0;
    do {
      v.push_back(zolo_step(l, rr));
      l = v.back().lnext;
    } while ((int)v.size() < cap && !(1.0 - l <= delta));
    ok = 1.0 - l <= delta;
    return v;
  };
  bool ok = false;
  if (r > 0) {
    std::vector<ZoloStep> v = run(r, max_steps, ok);
    return ok ? v : std::vector<ZoloStep>();
  }
  for (int rr = 1; rr <= 8; ++rr) {
    std::vector<ZoloStep> v = run(rr, 2, ok);
    if (ok) return v;
  }
  std::vector<ZoloStep> v = run(8, max_steps, ok);
  return ok ? v : std::vector<ZoloStep>();
}

}  // namespace hq

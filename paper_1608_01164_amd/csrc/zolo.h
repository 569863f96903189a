// Coefficients of the scaled Zolotarev functions behind Zolo-pd, the polar decomposition in a
// fixed small number of steps by Zolotarev's best rational approximations of the sign function
// (cited in Sec. 2.1 of the paper; Nakatsukasa and Freund, SIAM Review 58 (2016)).
#pragma once
#include <vector>

namespace hq {

// Type (2r+1, 2r) approximation on [l, 1]:
//   Zhat(x) = mhat x prod_j (x^2 + c[2j]) / (x^2 + c[2j-1])
//           = mhat (x + sum_j a[j] x / (x^2 + c[2j-1]))              (j = 1..r),
// with c_i = l^2 sc^2(i K' / (2r+1); l') (modulus l' = sqrt(1 - l^2), K' = K(l')), a_j > 0 the
// residues of the partial fractions, and mhat = prod_j (1 + c[2j-1]) / (1 + c[2j]) so that
// Zhat(1) = 1.  lnext = Zhat(l), the smallest value of Zhat on [l, 1].  Arrays are 1-based:
// c[1..2r], a[1..r] (index 0 unused).
struct ZoloStep {
  int r = 0;
  double l = 0, mhat = 0, lnext = 0;
  std::vector<double> c, a;
};

// One step's coefficients for l in [1e-150, 1) and 1 <= r <= 16; throws std::invalid_argument
// outside.  The Jacobi functions of modulus l' (close to 1 when l is small) are evaluated through
// Jacobi's imaginary transformation, sc(u | 1 - l^2) = -i sn(iu | l^2), with the arithmetic-
// geometric mean in the form where every quantity stays real (sinh / asinh in place of sin / asin),
// so the tiny complementary modulus l enters directly and no 1 - l^2 is ever rounded.
ZoloStep zolo_step(double l, int r);

// Schedule: the steps from l0 until 1 - l_k <= delta.  r = 0 picks the smallest r <= 8 that needs
// at most two steps (the method's design point), else r = 8 with as many steps as it takes (at most
// max_steps; an empty vector when that is not enough).
std::vector<ZoloStep> zolo_schedule(double l0, double delta, int r, int max_steps);

// Complete elliptic integral K(k') for the complementary modulus k' = sqrt(1 - l^2), from l.
double ellipk_complement(double l);
// sc(u | 1 - l^2) for 0 <= u <= K(sqrt(1 - l^2)).
double jacobi_sc_complement(double u, double l);

}  // namespace hq

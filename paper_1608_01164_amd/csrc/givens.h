// Structured QR of [c*(A - shift I); I] for symmetric b-banded A (Sec. 4 of the paper) and the
// HODLR factors of its orthogonal factor.
#pragma once
#include <cstdint>
#include <vector>

namespace hq {

struct Tree;

struct Rot {
  int64_t p, q;  // Q columns p, q:  Q[:,p] <- c Q[:,p] + s Q[:,q],  Q[:,q] <- -s Q[:,p] + c Q[:,q]
  double c, s;
};

struct GivensSweep {
  std::vector<Rot> rots;
  std::vector<int64_t> step;  // rots of step i (0-based) are [step[i], step[i+1])
};

// Algorithms 1 (b = 1) and 2 (b > 1) on [scale*(A - shift I); I]; A in LAPACK lower band storage.
GivensSweep structured_qr(const double* ab, int64_t n, int b, int64_t ldab, double shift, double scale);

// Host image of a HODLR matrix in the device layout of HMat (leaves ldl x ldl, factors per level
// with leading dimension ldf[l] and capacity cap[l], block (p, s) at (2i + s) * ldf * cap).
struct HostHodlr {
  std::vector<double> leaves;
  std::vector<std::vector<double>> U, V;
  std::vector<int> rank;
};

// Q1 = Q(0:n, 0:n) and Q2 = Q(n:2n, 0:n) of the sweep, directly in HODLR form: Q1 upper blocks have
// rank <= 2b, lower blocks rank b (b-Hessenberg corner); Q2 upper blocks rank <= 2b, lower ones 0.
void q_factors_hodlr(const GivensSweep& g, const Tree& t, int b, const std::vector<int>& cap, int ldl,
                     HostHodlr& q1, HostHodlr& q2);

}  // namespace hq

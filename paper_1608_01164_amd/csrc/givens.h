// Structured QR of [c*(A - shift I); I] for symmetric b-banded A (Sec. 4 of the paper) and the
// HODLR factors of its orthogonal factor.
#pragma once
#include <cstddef>
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
// with leading dimension ldf[l] and capacity cap[l], block (p, s) at (2i + s) * ldf * cap), as
// pointers into one block of doubles: caller-provided memory (pinned, for a direct copy to the
// device) or the object's own.
struct HostHodlr {
  double* leaves = nullptr;
  std::vector<double*> U, V;  // per level
  std::vector<size_t> fsize;  // doubles per level in U[l] (and in V[l])
  size_t nleaves = 0;         // doubles in leaves
  std::vector<int> rank;
  std::vector<double> own;
};

// Doubles one host image takes.
size_t host_hodlr_doubles(const Tree& t, const std::vector<int>& cap, int ldl);

// Q1 = Q(0:n, 0:n) and Q2 = Q(n:2n, 0:n) of the sweep, directly in HODLR form: Q1 upper blocks have
// rank <= 2b, lower blocks rank b (b-Hessenberg corner); Q2 upper blocks rank <= 2b, lower ones 0.
// mem, when given, holds 2 * host_hodlr_doubles(t, cap, ldl) doubles (Q1's image, then Q2's); every
// one of them is written.  Otherwise the images own their storage.
void q_factors_hodlr(const GivensSweep& g, const Tree& t, int b, const std::vector<int>& cap, int ldl,
                     HostHodlr& q1, HostHodlr& q2, double* mem = nullptr);

// structured_qr, then q_factors_hodlr on its sweep.  Returns the number of rotations.
int64_t q_factors_from_band(const double* ab, int64_t n, int b, int64_t ldab, double shift, double scale,
                            const Tree& t, const std::vector<int>& cap, int ldl, HostHodlr& q1, HostHodlr& q2,
                            double* mem = nullptr);

}  // namespace hq

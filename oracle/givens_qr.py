"""Dense reference for the fast QR decomposition of [A; I] -- TEST INFRASTRUCTURE.

Follows Sec. 4 of the paper: Algorithm 1 (tridiagonal A) and Algorithm 2 (banded A, b > 1).
R starts as [A; I] (2n x n) and Q as I_{2n}; every rotation G(p, q) is chosen to annihilate one
entry of R and is applied as R <- G^T R (rows p, q) and Q <- Q G (columns p, q), exactly in the
order the algorithms list them.  Everything is dense, O(n^2) memory: small n only.

The order of annihilation in step i (1-based):
  alpha_{i,i}: rows (n+1, n+i) zero R(n+i, i) against R(n+1, i)      [i >= 2]
  alpha_{i,j}: rows (n+i, n+j) zero R(n+i, j) against R(n+j, j),  j = i+1 .. min(n, b+i-1)
  beta_i     : rows (i, n+1)   zero R(n+1, i) against R(i, i)
  gamma_{i,j}: rows (i, j)     zero R(j, i)   against R(i, i),    j = i+1 .. min(n, b+i)   [i < n]
(step 1 has only beta_1 and the gammas).  For b = 1 this is exactly Algorithm 1.

Pinned by (tests/test_oracle_givens.py): the rotation counts 3n-2 and (2b+1)n - b^2 - b stated in
Sec. 4; [A; I] = Q R with Q orthogonal and R upper triangular (checked against numpy's QR through
R^T R = A^T A + I); Q1 b-Hessenberg and Q2 upper triangular; the rank bounds of Theorems
ranks_tridiag / ranks_banded / rank_tridiag_product; and the identity
Q1 Q2^T = sqrt(c) X (I + c X^T X)^{-1} for [sqrt(c) X; I] (independent of rotation signs).
"""
from __future__ import annotations

import numpy as np


def _rotation(f: float, g: float):
    r = float(np.hypot(f, g))
    if r == 0.0:
        return 1.0, 0.0
    return f / r, g / r


def fast_qr(A: np.ndarray, b: int):
    """Return (Q, R, rotations) for [A; I]; rotations is a list of (p, q, c, s) with 0-based rows.

    Row p is the pivot row, row q the row whose entry is annihilated.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    R = np.vstack([A.copy(), np.eye(n)])
    Q = np.eye(2 * n)
    rots = []

    def rot(p: int, q: int, col: int):
        c, s = _rotation(R[p, col], R[q, col])
        rp, rq = R[p, :].copy(), R[q, :].copy()
        R[p, :] = c * rp + s * rq
        R[q, :] = -s * rp + c * rq
        R[q, col] = 0.0
        qp, qq = Q[:, p].copy(), Q[:, q].copy()
        Q[:, p] = c * qp + s * qq
        Q[:, q] = -s * qp + c * qq
        rots.append((p, q, c, s))

    N1 = n  # 0-based index of row n+1
    # step 1
    rot(0, N1, 0)                                   # beta_1
    for j in range(1, min(n - 1, b) + 1):           # gamma_{1,j}, j = 2..b+1 (1-based)
        rot(0, j, 0)
    for i in range(1, n):                           # 0-based i  <->  paper's i+1
        rot(N1, n + i, i)                           # alpha_{i,i}
        for j in range(i + 1, min(n - 1, b + i - 1) + 1):
            rot(n + j, n + i, j)                    # alpha_{i,j}: pivot row n+j, zero R(n+i, j)
        rot(i, N1, i)                               # beta_i
        if i < n - 1:
            for j in range(i + 1, min(n - 1, b + i) + 1):
                rot(i, j, i)                        # gamma_{i,j}
    return Q, R, rots


def q1q2_product(X: np.ndarray, c: float, b: int):
    """Q1 Q2^T of the QR of [sqrt(c) X; I] by Algorithm 1/2, and the Q factors."""
    n = X.shape[0]
    Q, R, rots = fast_qr(np.sqrt(c) * X, b)
    Q1 = Q[:n, :n]
    Q2 = Q[n:, :n]
    return Q1 @ Q2.T, Q1, Q2, R, rots


def rotation_count(n: int, b: int) -> int:
    """The count the paper states: 3n - 2 for b = 1, (2b+1) n - b^2 - b for b > 1."""
    return 3 * n - 2 if b == 1 else (2 * b + 1) * n - b * b - b

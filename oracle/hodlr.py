"""Plain reader for a HODLR matrix exported by the library -- TEST INFRASTRUCTURE.

A HODLR matrix (Sec. 3.1.1, eq. HODLR) is given here as a plain dict of host arrays:
  n        -- order
  leaves   -- list of (lo, hi, D) with D the dense diagonal block rows/cols [lo, hi)
  blocks   -- list of (lo, mid, hi, Uu, Vu, Ul, Vl): the node [lo, hi) split at mid has the
              upper off-diagonal block M[lo:mid, mid:hi] = Uu Vu^T and the lower one
              M[mid:hi, lo:mid] = Ul Vl^T (factors may have zero columns).
The functions below assemble or apply it with nothing but slicing and matrix products, so
that a GPU result can be compared with the oracle's dense projector without trusting any of
the library's own arithmetic.  Pinned by tests/test_oracle_hodlr.py (compression of a known
dense matrix by numpy SVD reassembles to it; matvec equals dense @ x).
"""
from __future__ import annotations

import numpy as np


def to_dense(H: dict) -> np.ndarray:
    n = H["n"]
    M = np.zeros((n, n))
    for lo, hi, D in H["leaves"]:
        M[lo:hi, lo:hi] = D
    for lo, mid, hi, Uu, Vu, Ul, Vl in H["blocks"]:
        M[lo:mid, mid:hi] = Uu @ Vu.T
        M[mid:hi, lo:mid] = Ul @ Vl.T
    return M


def matvec(H: dict, X: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    Y = np.zeros_like(X)
    for lo, hi, D in H["leaves"]:
        Y[lo:hi] += D @ X[lo:hi]
    for lo, mid, hi, Uu, Vu, Ul, Vl in H["blocks"]:
        Y[lo:mid] += Uu @ (Vu.T @ X[mid:hi])
        Y[mid:hi] += Ul @ (Vl.T @ X[lo:mid])
    return Y


def trace(H: dict) -> float:
    return float(sum(np.trace(D) for _, _, D in H["leaves"]))


def compress_dense(M: np.ndarray, leaf: int, tol: float) -> dict:
    """HODLR approximation of a dense matrix by truncated SVDs of the off-diagonal blocks (Sec. 3.1.1)."""
    n = M.shape[0]
    leaves, blocks = [], []

    def rec(lo, hi):
        if hi - lo <= leaf:
            leaves.append((lo, hi, M[lo:hi, lo:hi].copy()))
            return
        mid = lo + (hi - lo + 1) // 2
        fac = []
        for blk in (M[lo:mid, mid:hi], M[mid:hi, lo:mid]):
            U, s, Vt = np.linalg.svd(blk, full_matrices=False)
            k = int(np.sum(s > tol))
            fac += [U[:, :k] * s[:k], Vt[:k].T]
        blocks.append((lo, mid, hi, *fac))
        rec(lo, mid)
        rec(mid, hi)

    rec(0, n)
    return {"n": n, "leaves": leaves, "blocks": blocks}

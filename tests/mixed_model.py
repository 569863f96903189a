"""Dense CPU model of the mixed-precision mode, used to state its error level in advance (tests only).

The QDWH iteration in its Cholesky form (eq. qdwh_chol_reccur), X_{k+1} = (b/c) X + (a - b/c) Y W^{-T}
with W^T W = I + c X^T X and Y W = X, is run densely with numpy.  After every iteration each off-
diagonal block of the cluster tree (split [lo, hi) at lo + ceil((hi - lo)/2) down to the leaf size) is
truncated by its SVD, as a HODLR recompression does.  Iterations marked FP32 form Z and the solves in
float32 (the Cholesky factorisation itself in float64, as the library's leaves) and truncate every
block at max(tol, floor(m) sigma_1), floor(m) the FP32 noise level of a block with m rows; the
others run in float64 and truncate at tol.  It models what the mixed mode does to the projector, not
how the library computes it: no code is shared with the HIP path.
"""
from __future__ import annotations

import numpy as np

from oracle import qdwh

U32 = 2.0 ** -24
TOL_AFTER_FP32 = 1e-8   # the library's truncation of FP64 iterations after FP32 ones (at least tol)


def floor_sqrt_m(m: int) -> float:
    """The library's FP32 truncation level of a block with m rows (relative to its sigma_1)."""
    return 4.0 * U32 * np.sqrt(max(m, 1))


def blocks(n: int, leaf: int):
    """(row range, column range) of every off-diagonal block of the cluster tree."""
    out = []
    stack = [(0, n)]
    while stack:
        lo, hi = stack.pop()
        if hi - lo <= leaf:
            continue
        mid = lo + (hi - lo + 1) // 2
        out.append(((lo, mid), (mid, hi)))
        out.append(((mid, hi), (lo, mid)))
        stack += [(lo, mid), (mid, hi)]
    return out


def truncate(X: np.ndarray, leaf: int, tol: float, floor=None) -> None:
    for (r0, r1), (c0, c1) in blocks(X.shape[0], leaf):
        B = X[r0:r1, c0:c1]
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        th = tol if floor is None else max(tol, floor(max(r1 - r0, c1 - c0)) * (s[0] if s.size else 0.0))
        k = int(np.count_nonzero(s > th))
        X[r0:r1, c0:c1] = (U[:, :k] * s[:k]) @ Vt[:k]


def certified_l0(lam: np.ndarray, mu: float, alpha: float) -> float:
    """The largest alpha 2^-j with no eigenvalue within it of mu, over alpha (the library's reading)."""
    dist = float(np.min(np.abs(lam - mu)))
    j = 0
    while alpha * 2.0 ** -j >= dist:
        j += 1
    return 2.0 ** -j


def fp32_iterations(sched, c_max: float = 16.0):
    K = len(sched)
    return [k for k in range(K) if 0 < k < K - 1 and sched[k][2] <= c_max]


def mixed_projector(A: np.ndarray, mu: float, lam: np.ndarray, leaf: int, tol: float, floor=floor_sqrt_m,
                    fp32: bool = True):
    """Projector of the dense model, its schedule and the iterations run in FP32."""
    n = A.shape[0]
    M = A - mu * np.eye(n)
    alpha = float(np.abs(M).sum(1).max())
    sched, _ = qdwh.schedule(certified_l0(lam, mu, alpha))
    f32 = fp32_iterations(sched) if fp32 else []
    X = M / alpha
    for k, (a, b, c, _l) in enumerate(sched):
        lowp = k in f32
        after = any(j < k for j in f32)
        dt = np.float32 if lowp else np.float64
        Xl = X.astype(dt)
        Z = np.eye(n, dtype=dt) + dt(c) * (Xl.T @ Xl)
        W = np.linalg.cholesky(Z.astype(np.float64)).T.astype(dt)  # W^T W = Z, W upper
        Y = np.linalg.solve(W.T, Xl.T).T      # Y W = X
        V = np.linalg.solve(W, Y.T).T         # V W^T = Y
        X = ((b / c) * Xl + dt(a - b / c) * V).astype(np.float64)
        truncate(X, leaf, max(tol, TOL_AFTER_FP32) if after and not lowp else tol, floor if lowp else None)
    P = 0.5 * (np.eye(n) - 0.5 * (X + X.T))
    return P, sched, f32


def stated_bound(n: int, sched, f32) -> float:
    """Error level of the mixed mode stated before any run.  An FP32 iteration k perturbs X_{k+1} by
    (i) the truncation of its largest blocks at floor(ceil(n/2)) sigma_1 (sigma_1 of a block of X is at
    most ||X|| <= 1) and (ii) the rounding noise of its FP32 products and Householder steps, about
    u32 sqrt(m) = floor / 4 each for the four formatted products of the iteration: together at most
    2 floor(ceil(n/2)).  The part of that perturbation that couples the eigenvectors on the two sides of
    mu is not undone by later iterations, which converge to the sign of the perturbed iterate; the
    eigenvalues of X_{k+1} are at least l_{k+1} away from 0, so the coupling turns the invariant
    subspace by at most about (perturbation) / (2 l_{k+1}) (Davis-Kahan).  Summed over the FP32
    iterations: sum_k floor(ceil(n/2)) / l_{k+1}.  The FP64 iterations after them truncate at
    TOL_AFTER_FP32 per block, at most levels x TOL_AFTER_FP32 on X_{k+1}, turned into a rotation the
    same way (l_{k+1} is near 1 by then)."""
    ls = [s[3] for s in sched] + [1.0]
    levels = max(1, int(np.ceil(np.log2(max(n, 2)))))
    post = [k for k in range(len(sched)) if f32 and k > min(f32) and k not in f32]
    return float(sum(2.0 * floor_sqrt_m((n + 1) // 2) / (2.0 * min(1.0, ls[k + 1])) for k in f32) +
                 sum(levels * TOL_AFTER_FP32 / (2.0 * min(1.0, ls[k + 1])) for k in post))


def bound_from_info(n: int, info: dict) -> float:
    """stated_bound for a solve, from the l0 and the FP32 iterations the library reports."""
    sched, _ = qdwh.schedule(info["l0"])
    return stated_bound(n, sched, [k for k, f in enumerate(info["fp32_iter"]) if f])

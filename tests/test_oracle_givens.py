"""Pins of the dense reference for the fast QR of [A; I] (Algorithms 1 and 2), CPU only."""
import numpy as np
import pytest

import workloads as w
from oracle import givens_qr as g


def _mat(n, b, seed):
    ab = w.tridiag_uniform(n, seed) if b == 1 else w.banded_normal(n, b, seed)
    return w.band_to_dense(ab)


@pytest.mark.parametrize("n,b", [(2, 1), (3, 1), (10, 1), (33, 1), (5, 2), (17, 2), (24, 3), (40, 4), (50, 8)])
def test_counts_structure_ranks(n, b):
    A = _mat(n, b, n + b)
    Q, R, rots = g.fast_qr(A, b)
    assert len(rots) == g.rotation_count(n, b)
    M = np.vstack([A, np.eye(n)])
    assert np.abs(Q @ R - M).max() < 1e-13
    assert np.abs(Q.T @ Q - np.eye(2 * n)).max() < 1e-13
    assert np.abs(np.tril(R[:n], -1)).max() == 0.0 and np.abs(R[n:]).max() == 0.0
    # R agrees with numpy's QR up to row signs: R^T R = A^T A + I
    assert np.abs(R[:n].T @ R[:n] - (A.T @ A + np.eye(n))).max() < 1e-12 * max(1, np.abs(A).max() ** 2)
    Q1, Q2 = Q[:n, :n], Q[n:, :n]
    assert np.abs(np.tril(Q1, -b - 1)).max() == 0.0          # b-Hessenberg
    assert np.abs(np.tril(Q2, -1)).max() == 0.0              # upper triangular
    for k in range(1, n):                                    # Theorems ranks_tridiag / ranks_banded
        assert np.linalg.matrix_rank(Q[:k, k:n], 1e-10) <= 2 * b
        assert np.linalg.matrix_rank(Q[n:n + k, k:n], 1e-10) <= 2 * b


@pytest.mark.parametrize("n,b,c", [(30, 1, 2.5), (64, 1, 1e4), (40, 3, 7.0), (48, 5, 1e6)])
def test_product_identity_and_ranks(n, b, c):
    X = _mat(n, b, 3)
    X = X / np.abs(np.linalg.eigvalsh(X)).max()
    P, Q1, Q2, R, _ = g.q1q2_product(X, c, b)
    ref = np.sqrt(c) * X @ np.linalg.inv(np.eye(n) + c * X.T @ X)
    assert np.abs(P - ref).max() < 1e-12 * max(1.0, np.sqrt(c))
    for k in range(1, n):                                    # Theorems rank_*_product
        assert np.linalg.matrix_rank(P[:k, k:], 1e-9) <= 2 * b
        assert np.linalg.matrix_rank(P[k:, :k], 1e-9) <= 2 * b
    if b == 1:                                               # X1 exactly rank <= 3 off the diagonal
        a0, b0, c0 = 10.0, 20.25, c
        X1 = (b0 / c0) * X + (1 / np.sqrt(c0)) * (a0 - b0 / c0) * P
        for k in range(1, n):
            assert np.linalg.matrix_rank(X1[k:, :k], 1e-9) <= 3

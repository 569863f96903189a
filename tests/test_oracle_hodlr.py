"""Pins of the oracle's HODLR reader and norm estimator (CPU only)."""
import numpy as np

from oracle import hodlr, norms


def test_compress_roundtrip_and_matvec():
    n = 333
    x = np.linspace(0, 1, n)
    K = np.exp(-np.abs(x[:, None] - x[None, :]))
    H = hodlr.compress_dense(K, 40, 1e-13)
    assert np.abs(hodlr.to_dense(H) - K).max() < 1e-12
    X = np.random.default_rng(0).standard_normal((n, 4))
    assert np.abs(hodlr.matvec(H, X) - K @ X).max() < 1e-11
    assert abs(hodlr.trace(H) - np.trace(K)) < 1e-12


def test_lanczos_norm():
    rng = np.random.default_rng(1)
    for n in (10, 200):
        A = rng.standard_normal((n, n))
        S = A + A.T
        assert abs(norms.lanczos_norm(lambda v: S @ v, n) - np.linalg.norm(S, 2)) < 1e-10 * np.linalg.norm(S, 2)

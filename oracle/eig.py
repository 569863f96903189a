"""Oracle spectral projector Pi_{<mu}(A) = sum_{lambda_i < mu} v_i v_i^T -- TEST INFRASTRUCTURE.

Definition followed: Sec. 1 of the paper (the problem statement) -- for a symmetric banded A
with lambda_1 <= ... <= lambda_nu < mu < lambda_{nu+1} <= ... <= lambda_n, the projector onto
the invariant subspace of the nu eigenvalues below mu.  Eigenvalues come from Sylvester-inertia
bisection, eigenvectors from inverse iteration (C core, eig_band.c), and Pi = V V^T is formed by a
plain matrix product.

Pinned by (tests/test_oracle_eig.py): numpy eigvalsh/eigh on small cases (library routine),
the closed-form projector of the 1D Laplacian (Sec. 6, Laplace example; entries through a
Dirichlet-kernel sum), the prescribed-spectrum generator of Sec. 6.1, and the invariants
Pi^2 = Pi, trace Pi = nu, ||A Pi - Pi A|| <= 1e-12 ||A||.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_count.restype = ctypes.c_long
        L.oracle_count.argtypes = [ctypes.c_long, ctypes.c_int, dp, ctypes.c_long, ctypes.c_double,
                                   ctypes.c_double, dp]
        L.oracle_bisect.restype = None
        L.oracle_bisect.argtypes = [ctypes.c_long, ctypes.c_int, dp, ctypes.c_long, ctypes.c_long,
                                    ctypes.c_long, dp]
        L.oracle_inverse_iteration.restype = None
        L.oracle_inverse_iteration.argtypes = [ctypes.c_long, ctypes.c_int, dp, ctypes.c_long, ctypes.c_long,
                                               dp, ctypes.c_long, dp]
        L.oracle_window_mgs.restype = None
        L.oracle_window_mgs.argtypes = [ctypes.c_long, ctypes.c_long, dp, ctypes.c_double, dp]
        L.oracle_norm_inf.restype = ctypes.c_double
        L.oracle_norm_inf.argtypes = [ctypes.c_long, ctypes.c_int, dp, ctypes.c_long]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_band(ab: np.ndarray):
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    if ab.ndim != 2:
        raise ValueError("band must be (n, ld)")
    return ab


def bandwidth(ab: np.ndarray) -> int:
    n, ld = ab.shape
    b = 0
    for i in range(1, ld):
        if np.any(ab[: n - i, i] != 0.0):
            b = i
    return max(b, 1)


def norm_inf(ab: np.ndarray) -> float:
    ab = _check_band(ab)
    n, ld = ab.shape
    return float(lib().oracle_norm_inf(n, bandwidth(ab), _p(ab), ld))


def count(ab: np.ndarray, sigma: float) -> int:
    """#{lambda_i < sigma}: negative pivots of the LDL^T of A - sigma I (Sylvester's law of inertia)."""
    ab = _check_band(ab)
    n, ld = ab.shape
    b = bandwidth(ab)
    pivmin = np.finfo(np.float64).tiny * max(1.0, float(np.max(ab[:, 1:] ** 2)) if ld > 1 else 1.0)
    return int(lib().oracle_count(n, b, _p(ab), ld, float(sigma), pivmin, None))


def eigenvalues(ab: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """lambda_{k0} .. lambda_{k1} (1-based, inclusive), ascending, by bisection."""
    ab = _check_band(ab)
    n, ld = ab.shape
    out = np.empty(k1 - k0 + 1)
    lib().oracle_bisect(n, bandwidth(ab), _p(ab), ld, k0, k1, _p(out))
    return out


def midpoint_shift(ab: np.ndarray, nu: int):
    """mu = (lambda_nu + lambda_{nu+1}) / 2 and the gap lambda_{nu+1} - lambda_nu."""
    lam = eigenvalues(ab, nu, nu + 1)
    return 0.5 * (lam[0] + lam[1]), float(lam[1] - lam[0]), lam


def eigenvectors(ab: np.ndarray, lam: np.ndarray, seed: int = 0, ortol_rel: float = 1e-3) -> np.ndarray:
    """Columns v_k for the (ascending) eigenvalues lam: inverse iteration, then windowed MGS."""
    ab = _check_band(ab)
    n, ld = ab.shape
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    m = lam.size
    V = np.empty((m, n))        # row k = v_k, i.e. column-major n x m
    lib().oracle_inverse_iteration(n, bandwidth(ab), _p(ab), ld, m, _p(lam), seed, _p(V))
    lib().oracle_window_mgs(n, m, _p(lam), ortol_rel * norm_inf(ab), _p(V))
    return V.T                  # n x m view


def band_matvec(ab: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x for the symmetric band matrix (x may be n x k)."""
    n, ld = ab.shape
    x = np.asarray(x, dtype=np.float64)
    y = ab[:, 0].reshape((n,) + (1,) * (x.ndim - 1)) * x
    for i in range(1, ld):
        c = ab[: n - i, i].reshape((n - i,) + (1,) * (x.ndim - 1))
        y[i:] += c * x[: n - i]
        y[: n - i] += c * x[i:]
    return y


class Projector:
    """Pi = V V^T for the eigenvalues below mu (dense Pi optional)."""

    def __init__(self, ab, mu, nu, lam, V, gap, timings):
        self.ab, self.mu, self.nu, self.lam, self.V, self.gap, self.timings = ab, mu, nu, lam, V, gap, timings
        self._Pi = None

    @property
    def Pi(self) -> np.ndarray:
        if self._Pi is None:
            self._Pi = self.V @ self.V.T
        return self._Pi

    def apply(self, X: np.ndarray) -> np.ndarray:
        return self.V @ (self.V.T @ X)

    def invariants(self) -> dict:
        """||V^T V - I||_max, |trace - nu|, ||A V - V Lambda||_F / ||A||_inf, ||Pi^2 - Pi||_max."""
        V = self.V
        G = V.T @ V
        res = band_matvec(self.ab, V) - V * self.lam[None, :]
        anorm = norm_inf(self.ab)
        out = {
            "orth": float(np.max(np.abs(G - np.eye(G.shape[0])))),
            "trace_err": float(abs(np.sum(V * V) - self.nu)),
            "residual_rel": float(np.linalg.norm(res) / anorm),
        }
        if V.shape[0] <= 4096:
            P = self.Pi
            out["idem"] = float(np.max(np.abs(P @ P - P)))
            AP = band_matvec(self.ab, P)
            out["commute_rel"] = float(np.linalg.norm(AP - AP.T, 2) / anorm)
        return out


def spectral_projector(ab: np.ndarray, nu: int | None = None, mu: float | None = None, seed: int = 0) -> Projector:
    """Oracle Pi_{<mu}(A).  Give nu (mu := midpoint of lambda_nu, lambda_{nu+1}) or mu (nu := count(mu))."""
    ab = _check_band(ab)
    n = ab.shape[0]
    t = {}
    t0 = time.perf_counter()
    if mu is None:
        if nu is None:
            nu = n // 2
        mu, gap, _ = midpoint_shift(ab, nu)
    else:
        nu = count(ab, mu)
        gap = float("nan")
        if 0 < nu < n:
            l2 = eigenvalues(ab, nu, nu + 1)
            gap = float(l2[1] - l2[0])
    t["shift"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    lam = eigenvalues(ab, 1, nu) if nu > 0 else np.zeros(0)
    t["bisection"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    V = eigenvectors(ab, lam, seed=seed) if nu > 0 else np.zeros((n, 0))
    t["inverse_iteration"] = time.perf_counter() - t0
    return Projector(ab, float(mu), int(nu), lam, V, gap, t)


def num_threads() -> int:
    return int(lib().oracle_num_threads())

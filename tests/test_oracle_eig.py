"""Pins of the oracle projector (CPU only): it must agree with things other than itself."""
import math

import numpy as np
import pytest

import workloads as w
from oracle import eig


def laplace_projector(n: int, nu: int) -> np.ndarray:
    """Closed form: eigenvectors sqrt(2/(n+1)) sin(jk theta), theta = pi/(n+1), of tridiag(-1,0,-1)
    with eigenvalues -2cos(k theta) (paper Sec. 6.2).  Summing the nu lowest,
    Pi_jl = (1/(n+1)) [D(j-l) - D(j+l)], D(x) = sum_{k=1}^{nu} cos(k x theta)."""
    th = math.pi / (n + 1)
    j = np.arange(1, n + 1)
    diff = (j[:, None] - j[None, :]) * th
    summ = (j[:, None] + j[None, :]) * th

    def D(x):
        out = np.empty_like(x)
        s = np.sin(x / 2)
        small = np.abs(s) < 1e-14
        out[~small] = np.sin(nu * x[~small] / 2) * np.cos((nu + 1) * x[~small] / 2) / s[~small]
        # x a multiple of 2*pi: every cosine is +-1
        out[small] = nu * np.cos(x[small] / 2 * 0)  # cos(k*2pi m) = 1
        return out

    return (D(diff) - D(summ)) / (n + 1)


@pytest.mark.parametrize("n", [8, 64, 257, 1000])
def test_laplace_closed_form(n):
    nu = n // 2
    ab = w.laplacian(n)
    P = eig.spectral_projector(ab, nu=nu)
    lam_exact = -2 * np.cos(np.arange(1, nu + 1) * math.pi / (n + 1))
    assert np.max(np.abs(P.lam - lam_exact)) < 1e-13
    ref = laplace_projector(n, nu)
    assert np.max(np.abs(P.Pi - ref)) < 1e-12 * max(1, n / 100)
    # the oracle's gap equals the exact middle gap
    assert abs(P.gap - (2 * np.cos((nu) * math.pi / (n + 1)) - 2 * np.cos((nu + 1) * math.pi / (n + 1)))) < 1e-13


@pytest.mark.parametrize("n,b,seed", [(2, 1, 0), (5, 1, 1), (7, 2, 2), (8, 3, 3), (8, 7, 4)])
def test_brute_force_tiny(n, b, seed):
    ab = w.banded_normal(n, b, seed)
    A = w.band_to_dense(ab)
    lam, V = np.linalg.eigh(A)
    for nu in range(1, n):
        P = eig.spectral_projector(ab, nu=nu)
        assert np.max(np.abs(P.Pi - V[:, :nu] @ V[:, :nu].T)) < 1e-12
        assert abs(P.mu - 0.5 * (lam[nu - 1] + lam[nu])) < 1e-12
    # counts at many shifts
    for s in np.linspace(lam[0] - 1, lam[-1] + 1, 41):
        assert eig.count(ab, s) == int(np.sum(lam < s))


@pytest.mark.parametrize("maker", [
    lambda: w.tridiag_uniform(600, 3), lambda: w.tridiag_metallic(500, 1),
    lambda: w.banded_normal(700, 4, 2), lambda: w.banded_normal(400, 16, 5)])
def test_counts_and_eigenvalues_vs_eigvalsh(maker):
    ab = maker()
    n = ab.shape[0]
    lam = np.linalg.eigvalsh(w.band_to_dense(ab))
    rng = np.random.default_rng(0)
    for s in rng.uniform(lam[0] - 0.5, lam[-1] + 0.5, 50):
        assert eig.count(ab, s) == int(np.sum(lam < s))
    got = eig.eigenvalues(ab, 1, n)
    assert np.max(np.abs(got - lam)) < 1e-11 * max(1.0, np.max(np.abs(lam)))


@pytest.mark.parametrize("b", [1, 2, 5])
def test_prescribed_spectrum(b):
    lam = w.split_gap_spectrum(120, 1e-3, seed=b)
    ab = w.prescribed_spectrum(lam, b)
    got = eig.eigenvalues(ab, 1, 120)
    assert np.max(np.abs(got - lam)) < 1e-13
    P = eig.spectral_projector(ab, nu=60)
    assert abs(P.mu) < 1e-3 and abs(P.gap - 2e-3) < 1e-13


@pytest.mark.parametrize("maker,nu", [
    (lambda: w.tridiag_uniform(1024, 0), 512), (lambda: w.banded_normal(1500, 8, 0), 750),
    (lambda: w.tridiag_metallic(2048, 0), 1024)])
def test_invariants(maker, nu):
    ab = maker()
    P = eig.spectral_projector(ab, nu=nu)
    inv = P.invariants()
    assert inv["orth"] < 1e-12
    assert inv["trace_err"] < 1e-9
    assert inv["idem"] < 1e-12
    assert inv["commute_rel"] < 1e-12
    assert eig.count(ab, P.mu) == nu


def test_full_projector_vs_eigh():
    ab = w.banded_normal(900, 3, 7)
    A = w.band_to_dense(ab)
    lam, V = np.linalg.eigh(A)
    P = eig.spectral_projector(ab, nu=300)
    assert np.linalg.norm(P.Pi - V[:, :300] @ V[:, :300].T, 2) < 1e-11

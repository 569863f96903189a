"""The Sec. 6.1 test-matrix generator in band storage (workloads/prescribed.c): the matrix it builds is
symmetric banded and orthogonally similar to diag(lambda), so its eigenvalues are the prescribed ones;
for a tridiagonal matrix it follows the dense construction's rotations exactly."""
import numpy as np
import pytest

import workloads as w


@pytest.mark.parametrize("n,b,gap", [(300, 1, 1e-3), (257, 3, 1e-6), (400, 8, 1e-1), (130, 16, 1e-4)])
def test_prescribed_band_has_the_prescribed_spectrum(n, b, gap):
    lam = w.split_gap_spectrum(n, gap, 3)
    ab = w.prescribed_spectrum_band(lam, b)
    A = w.band_to_dense(ab)
    ev = np.linalg.eigvalsh(A)
    assert np.abs(ev - np.sort(lam)).max() <= 1e-13
    # the first off-diagonal is populated (the outer ones decay with the distance from the diagonal:
    # the construction's fill in diagonal d is a product of d rotation sines)
    assert np.median(np.abs(ab[: n - 1, 1])) > 1e-3
    # exactly half the spectrum below 0, the gap at 0 as prescribed
    assert np.sum(ev < 0) == n // 2
    assert abs(ev[n // 2 - 1] + gap) <= 1e-13 and abs(ev[n // 2] - gap) <= 1e-13


def test_prescribed_band_matches_dense_construction_tridiagonal():
    lam = w.split_gap_spectrum(80, 1e-2, 5)
    # the same rotations in the same order; the two storages round the chase differently
    assert np.abs(w.prescribed_spectrum_band(lam, 1) - w.prescribed_spectrum(lam, 1)).max() <= 1e-12


def test_prescribed_band_large_order_runs_in_quadratic_time():
    import time
    lam = w.split_gap_spectrum(8000, 1e-4, 0)
    t = time.perf_counter()
    ab = w.prescribed_spectrum_band(lam, 4)
    assert time.perf_counter() - t < 20.0
    # trace and Frobenius norm are similarity invariants
    assert abs(ab[:, 0].sum() - lam.sum()) <= 1e-10
    fro2 = (ab[:, 0] ** 2).sum() + 2 * (ab[:, 1:] ** 2).sum()
    assert abs(fro2 - (lam ** 2).sum()) <= 1e-9 * (lam ** 2).sum()

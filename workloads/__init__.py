"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *draws* matrices.  It contains none of the spectral-projector
arithmetic, so that both the oracle and the HIP path can consume identical
inputs without sharing any code of the method.

Storage convention (both sides use it): a symmetric b-banded matrix A of order n
is held in LAPACK lower band storage, as a C-contiguous float64 array ``ab`` of
shape (n, ld) with ld >= b+1 and ``ab[j, i] = A(j+i, j)`` for 0 <= i <= b,
j+i < n (entries past the end of the matrix are zero).  Viewed as a flat buffer
this is column-major ``ab[i + j*ld]``, i.e. exactly LAPACK's ``dsbev`` lower
layout, so it crosses the C ABI without copies.

Workload families (seeded; shapes and value distributions of the paper's test problems):

* ``tridiag_uniform``   : diag ~ U(-2,2), off-diag ~ U(0.5,1)   (n=1024 and n=100000 runs)
* ``banded_normal``     : band entries N(0,1) mirrored, + 4*i/n on the diagonal
* ``tridiag_metallic``  : diag 2+v, v ~ U(0,0.1), off-diag -1    (small relative gap)
* ``laplacian``         : tridiag(-1, 0, -1), eigenvalues -2cos(k*pi/(n+1))
* ``batched_banded``    : many banded_normal matrices of uneven n and b
* ``prescribed_spectrum``: Sec. 6.1 of the paper -- a banded matrix with a given
  spectrum, built by Givens similarity plus bulge chasing (test matrices only).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "band_empty", "tridiag_uniform", "banded_normal", "tridiag_metallic", "laplacian",
    "batched_banded", "prescribed_spectrum", "band_to_dense", "dense_to_band",
    "split_gap_spectrum", "prescribed_spectrum_band", "build_native",
]


def band_empty(n: int, b: int, ld: int | None = None) -> np.ndarray:
    ld = b + 1 if ld is None else ld
    if ld < b + 1:
        raise ValueError("ld must be >= b+1")
    return np.zeros((n, ld), dtype=np.float64)


def tridiag_uniform(n: int, seed: int = 0) -> np.ndarray:
    """diag d_i ~ U(-2, 2), then off-diagonal e_i ~ U(0.5, 1) (draw order fixed)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-2.0, 2.0, n)
    e = rng.uniform(0.5, 1.0, n - 1)
    ab = band_empty(n, 1)
    ab[:, 0] = d
    ab[: n - 1, 1] = e
    return ab


def banded_normal(n: int, b: int, seed: int = 0, rng: np.random.Generator | None = None) -> np.ndarray:
    """Band entries (diagonal included) i.i.d. N(0,1), mirrored, plus 4*i/n on the diagonal, i=1..n.

    Superdiagonal j (j = 0..b) is drawn as ``standard_normal(n-j)`` in order j = 0, 1, ..., b.
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    ab = band_empty(n, b)
    for j in range(b + 1):
        ab[: n - j, j] = rng.standard_normal(n - j)
    ab[:, 0] += 4.0 * np.arange(1, n + 1, dtype=np.float64) / n
    return ab


def tridiag_metallic(n: int, seed: int = 0) -> np.ndarray:
    """diag 2 + v_i with v_i ~ U(0, 0.1), off-diagonal -1."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 0.1, n)
    ab = band_empty(n, 1)
    ab[:, 0] = 2.0 + v
    ab[: n - 1, 1] = -1.0
    return ab


def laplacian(n: int) -> np.ndarray:
    """tridiag(-1, 0, -1): the 1D Laplacian shifted by 2 (Sec. 6, 1D Laplace example)."""
    ab = band_empty(n, 1)
    ab[: n - 1, 1] = -1.0
    return ab


def batched_banded(count: int = 256, seed: int = 0, nmin: int = 2048, nmax: int = 16384,
                   bmax: int = 16):
    """``count`` banded_normal matrices with n_i ~ U{nmin..nmax}, b_i ~ U{1..bmax}.

    Sizes are drawn from ``default_rng(seed)``; matrix i then uses ``default_rng([seed, i])``.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    bs = rng.integers(1, bmax + 1, size=count)
    out = []
    for i in range(count):
        out.append(banded_normal(int(ns[i]), int(bs[i]), rng=np.random.default_rng([seed, i])))
    return out


def band_to_dense(ab: np.ndarray) -> np.ndarray:
    n, ld = ab.shape
    A = np.zeros((n, n))
    for i in range(ld):
        if i >= n:
            break
        idx = np.arange(n - i)
        A[idx + i, idx] = ab[: n - i, i]
        A[idx, idx + i] = ab[: n - i, i]
    return A


def dense_to_band(A: np.ndarray, b: int) -> np.ndarray:
    n = A.shape[0]
    ab = band_empty(n, b)
    for i in range(b + 1):
        idx = np.arange(n - i)
        ab[: n - i, i] = A[idx + i, idx]
    return ab


def split_gap_spectrum(n: int, gap: float, seed: int = 0) -> np.ndarray:
    """Eigenvalues uniform in [-1, -gap] U [gap, 1], half on each side (Sec. 6.1 experiments)."""
    rng = np.random.default_rng(seed)
    h = n // 2
    neg = -rng.uniform(gap, 1.0, h)
    pos = rng.uniform(gap, 1.0, n - h)
    neg[0] = -gap
    pos[0] = gap
    return np.sort(np.concatenate([neg, pos]))


def _rot(f: float, g: float):
    r = float(np.hypot(f, g))
    if r == 0.0:
        return 1.0, 0.0
    return f / r, g / r


def prescribed_spectrum(lams, b: int) -> np.ndarray:
    """Symmetric b-banded matrix orthogonally similar to diag(lams) (paper Sec. 6.1).

    For i = n, ..., 2 a plane rotation in (i-1, i) is chosen from the vector [a_ii, 1] and
    applied as a similarity; entries pushed outside the band are chased towards the bottom
    right corner with further plane rotations.  Dense O(n^3) -- test matrices of order a few
    hundred only.  Returns lower band storage.
    """
    lams = np.asarray(lams, dtype=np.float64)
    n = lams.size
    A = np.diag(lams.copy())

    def apply(p: int, q: int, c: float, s: float):
        # A <- G^T A G with G acting on coordinates (p, q): [c s; -s c] on rows, transposed on cols
        rp, rq = A[p, :].copy(), A[q, :].copy()
        A[p, :] = c * rp + s * rq
        A[q, :] = -s * rp + c * rq
        cp, cq = A[:, p].copy(), A[:, q].copy()
        A[:, p] = c * cp + s * cq
        A[:, q] = -s * cp + c * cq

    for i in range(n - 1, 0, -1):            # 0-based i <-> paper's i+1
        c, s = _rot(A[i, i], 1.0)
        apply(i - 1, i, c, s)
        # chase every entry that left the band, scanning down-right
        r = i - 1
        while True:
            cols = np.nonzero(np.abs(A[r, r + b + 1:]) > 0.0)[0]
            if cols.size == 0:
                break
            cc = r + b + 1 + int(cols[-1])   # outermost bulge entry in row r
            # annihilate A[r, cc] with a rotation of coordinates (cc-1, cc)
            c, s = _rot(A[r, cc - 1], A[r, cc])
            # rotation chosen so that the new A[r, cc] = -s*A[r,cc-1] + c*A[r,cc] = 0
            apply(cc - 1, cc, c, s)
            A[r, cc] = 0.0
            A[cc, r] = 0.0
            r = cc - 1
            if r + b + 1 >= n:
                break
    # everything outside the band is rounding noise now
    return dense_to_band(A, b)


# ---- Sec. 6.1 generator in band storage (C, O(n^2) flops) -------------------------------------

import ctypes as _ct
import os as _os
import subprocess as _sp

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_SO = _os.path.join(_HERE, "_prescribed.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile prescribed.c into workloads/_prescribed.so with gcc."""
    src = _os.path.join(_HERE, "prescribed.c")
    if not force and _os.path.exists(_SO) and _os.path.getmtime(_SO) >= _os.path.getmtime(src):
        return _SO
    tmp = _SO + ".tmp%d" % _os.getpid()
    _sp.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    _os.replace(tmp, _SO)
    return _SO


def prescribed_spectrum_band(lams, b: int) -> np.ndarray:
    """The Sec. 6.1 construction (same rotations as ``prescribed_spectrum``) carried out in band storage
    with one extra diagonal for the bulge: O(n^2) flops, for orders in the tens of thousands."""
    global _lib
    if _lib is None:
        _lib = _ct.CDLL(build_native())
        _lib.prescribed_band.restype = _ct.c_int
        _lib.prescribed_band.argtypes = [_ct.c_int64, _ct.c_int, _ct.c_void_p, _ct.c_void_p, _ct.c_int64]
    lams = np.ascontiguousarray(lams, dtype=np.float64)
    n = lams.size
    ab = band_empty(n, b)
    if _lib.prescribed_band(n, int(b), lams.ctypes.data, ab.ctypes.data, b + 1) != 0:
        raise MemoryError("prescribed_band: workspace")
    return ab

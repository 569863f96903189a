"""CPU pins of the mixed mode's stated error level (tests/mixed_model.py).

A dense model of the iteration with FP32 middle iterations and the library's FP32 truncation level
4 u32 sqrt(m) sigma_1 lands within a factor 10 below the stated bound, and the same model with the
level 8 u32 sigma_1 (no sqrt(m); the level of the survey's dense simulation) is several times more
accurate: the FP32 truncation level of the largest blocks is what sets the mixed mode's error.
"""
import numpy as np
import pytest

import workloads as w
from oracle import eig
from tests import mixed_model as mm

CASES = [
    ("tri-1024-leaf64", lambda: w.tridiag_uniform(1024, 0), 64),
    ("metallic-777-leaf64", lambda: w.tridiag_metallic(777, 2), 64),
]


@pytest.mark.parametrize("name,maker,leaf", CASES, ids=[c[0] for c in CASES])
def test_mixed_error_level(name, maker, leaf):
    ab = maker()
    n = ab.shape[0]
    ref = eig.spectral_projector(ab, nu=n // 2)
    A = w.band_to_dense(ab)
    lam = np.linalg.eigvalsh(A)
    P, sched, f32 = mm.mixed_projector(A, ref.mu, lam, leaf, 1e-10)
    err = np.linalg.norm(P - ref.Pi, 2)
    bound = mm.stated_bound(n, sched, f32)
    P8, _, _ = mm.mixed_projector(A, ref.mu, lam, leaf, 1e-10, floor=lambda m: 8 * mm.U32)
    err8 = np.linalg.norm(P8 - ref.Pi, 2)
    P64, _, _ = mm.mixed_projector(A, ref.mu, lam, leaf, 1e-10, fp32=False)
    err64 = np.linalg.norm(P64 - ref.Pi, 2)
    print(f"{name}: FP32 iterations {f32}; model error {err:.2e} (stated bound {bound:.2e}), "
          f"with the 8 u32 level {err8:.2e}, FP64 {err64:.2e}")
    assert f32
    assert bound / 10 <= err <= bound
    assert err8 <= err / 5
    assert err64 <= 1e-9

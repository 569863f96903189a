"""QDWH scalar schedule and exact-arithmetic iterate map -- TEST INFRASTRUCTURE.

Follows Sec. 2.1 of the paper (eq. qdwh_parameters_abc and the l_k recurrence):

    a_k = h(l_k),  b_k = (a_k - 1)^2 / 4,  c_k = a_k + b_k - 1,
    l_{k+1} = l_k (a_k + b_k l_k^2) / (1 + c_k l_k^2),
    h(l) = sqrt(1 + g) + 1/2 sqrt(8 - 4 g + 8 (2 - l^2) / (l^2 sqrt(1 + g))),  g = (4 (1 - l^2) / l^4)^(1/3),

iterating while |1 - l_k| > delta (Alg. 3).  The rational map of one step is
f_k(x) = x (a_k + b_k x^2) / (1 + c_k x^2) (eq. reccur restricted to an eigenvalue), so in exact
arithmetic X_K = V diag(f_{K-1} o ... o f_0 (lambda_i / alpha)) V^T.

Pinned by (tests/test_oracle_qdwh.py): h(1) = 3 so (a, b, c) = (3, 1, 3); f_k(1) = 1 from
c = a + b - 1; max of f_k on [l_k, 1] equals 1; at most six iterations for l_0 >= 1e-16 (the
kappa <= 1e16 claim of Sec. 2.1); c_k decreasing towards 3; the eigenvalue map driving every
|x| >= l_0 to within delta of sign(x).
"""
from __future__ import annotations

import math

import numpy as np


def h(l: float) -> float:
    l2 = l * l
    g = (4.0 * (1.0 - l2) / (l2 * l2)) ** (1.0 / 3.0)
    sg = math.sqrt(1.0 + g)
    return sg + 0.5 * math.sqrt(8.0 - 4.0 * g + 8.0 * (2.0 - l2) / (l2 * sg))


def weights(l: float):
    a = h(l)
    b = (a - 1.0) ** 2 / 4.0
    c = a + b - 1.0
    return a, b, c


def schedule(l0: float, delta: float = 1e-15, max_iter: int = 20):
    """List of (a_k, b_k, c_k, l_k) for k = 0 .. K-1, and the final l_K."""
    out = []
    l = float(l0)
    k = 0
    while abs(1.0 - l) > delta and k < max_iter:
        a, b, c = weights(l)
        out.append((a, b, c, l))
        l = l * (a + b * l * l) / (1.0 + c * l * l)
        k += 1
    return out, l


def f(x, a: float, b: float, c: float):
    x = np.asarray(x, dtype=np.float64)
    return x * (a + b * x * x) / (1.0 + c * x * x)


def iterate_eigenvalues(x, sched, upto: int | None = None):
    """Apply f_0, ..., f_{upto-1} to the scaled eigenvalues x = lambda / alpha."""
    x = np.asarray(x, dtype=np.float64).copy()
    steps = sched if upto is None else sched[:upto]
    for (a, b, c, _l) in steps:
        x = f(x, a, b, c)
    return x


def exact_iterate(lam, V, alpha: float, sched, upto: int | None = None) -> np.ndarray:
    """X_k = V diag(f_{k-1} o ... o f_0(lam / alpha)) V^T (full eigen-decomposition required)."""
    x = iterate_eigenvalues(np.asarray(lam) / alpha, sched, upto)
    return (V * x[None, :]) @ V.T

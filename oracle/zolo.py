"""Zolo-pd scalar schedule and exact-arithmetic iterate map -- TEST INFRASTRUCTURE.

Zolo-pd (the alternative to QDWH that Sec. 2.1 of the paper cites; Nakatsukasa and Freund, SIAM
Review 58, 2016) replaces the (3, 2) rational map of a QDWH step by the scaled Zolotarev function
of type (2r+1, 2r), the best rational approximation of sign(x) on [-1, -l] u [l, 1]:

    Zhat(x) = mhat x prod_{j=1..r} (x^2 + c_{2j}) / (x^2 + c_{2j-1}),
    c_i = l^2 sc^2(i K' / (2r+1); l'),  l' = sqrt(1 - l^2),  K' = K(l'),
    mhat = prod_j (1 + c_{2j-1}) / (1 + c_{2j})     (so that Zhat(1) = 1),

written for the matrix iteration in partial fractions,
    Zhat(x) = mhat (x + sum_j a_j x / (x^2 + c_{2j-1})),
    a_j = prod_k (c_{2k} - c_{2j-1}) / prod_{k != j} (c_{2k-1} - c_{2j-1}),
and the lower bound moves to l_next = Zhat(l).  With r = 8 two steps reach 1 - u from l = 1e-16.

The Jacobi function of modulus l' (close to 1 when l is small) is evaluated here from Jacobi's
theta series of the small modulus l at an imaginary argument (sc(w | l'^2) = -i sn(iw | l^2),
sn = theta3(0)/theta2(0) theta1/theta4 with nome q = exp(-pi K'/K)); the library takes a different
route (the arithmetic-geometric mean), so the two share no arithmetic.

Pinned by (tests/test_oracle_zolo.py): r = 1 reproduces the QDWH weights of eq.
qdwh_parameters_abc (c_1 = 1/c, c_2 = a/b, mhat = b/c); Zhat equioscillates on [l, 1] (r + 1 maxima
equal to 1 and r + 1 minima equal to Zhat(l), the defining property of the best approximation);
scipy's ellipj where 1 - l^2 is representable; the dense iteration reaching sign(A - mu I).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipk, ellipkm1


def _k_pair(l: float):
    """K = K(l) and K' = K(l') for the modulus l (parameter l^2), both accurate for tiny l."""
    return float(ellipk(l * l)), float(ellipkm1(l * l))


def sc_complement(w: float, l: float) -> float:
    """sc(w | 1 - l^2) for 0 <= w < K(l') by the theta series of modulus l at argument i w."""
    K, Kp = _k_pair(l)
    T = math.pi * Kp / K           # q = exp(-T)
    y = math.pi * w / (2.0 * K)    # x = i y
    nmax = 12

    def lsinh(x):  # log(sinh(x)), x > 0
        return x - math.log(2.0) + math.log1p(-math.exp(-2.0 * x))

    def lcosh(x):  # log(cosh(x)), x >= 0
        return x - math.log(2.0) + math.log1p(math.exp(-2.0 * x))

    def ex(v):  # exp without overflow warnings for the terms that vanish
        return math.exp(v) if v > -745.0 else 0.0

    # theta2(0), theta3(0) of nome q
    th2 = 2.0 * sum(ex(-T * (n + 0.5) ** 2) for n in range(nmax))
    th3 = 1.0 + 2.0 * sum(ex(-T * n * n) for n in range(1, nmax))
    # theta1(i y) / i and theta4(i y), each term as exp(log q^(...) + log sinh / cosh)
    t1 = 2.0 * sum((-1) ** n * ex(-T * (n + 0.5) ** 2 + lsinh((2 * n + 1) * y)) for n in range(nmax)) if y > 0 else 0.0
    t4 = 1.0 + 2.0 * sum((-1) ** n * ex(-T * n * n + lcosh(2 * n * y)) for n in range(1, nmax))
    return (th3 / th2) * t1 / t4


def step(l: float, r: int):
    """(c[1..2r], a[1..r], mhat, l_next) of one Zolo-pd step (lists 1-based, index 0 unused)."""
    _, Kp = _k_pair(l)
    c = [0.0] + [l * l * sc_complement(i * Kp / (2 * r + 1), l) ** 2 for i in range(1, 2 * r + 1)]
    a = [0.0]
    for j in range(1, r + 1):
        num = 1.0
        den = 1.0
        for k in range(1, r + 1):
            num *= c[2 * k] - c[2 * j - 1]
            if k != j:
                den *= c[2 * k - 1] - c[2 * j - 1]
        a.append(num / den)
    mhat = 1.0
    for j in range(1, r + 1):
        mhat *= (1.0 + c[2 * j - 1]) / (1.0 + c[2 * j])
    return c, a, mhat, min(1.0, float(zhat(l, c, mhat, r)))


def zhat(x, c, mhat, r):
    """The scaled Zolotarev function (product form)."""
    x = np.asarray(x, dtype=np.float64)
    f = mhat * x
    for j in range(1, r + 1):
        f = f * (x * x + c[2 * j]) / (x * x + c[2 * j - 1])
    return f


def schedule(l0: float, delta: float = 1e-15, r: int = 0, max_steps: int = 6):
    """Steps [(r, l_k, c, a, mhat)] from l0 until 1 - l_K <= delta (at least one step).  r = 0: the
    smallest r <= 8 that needs at most two steps, else r = 8 with up to max_steps steps."""
    def run(rr, cap):
        out, l = [], float(l0)
        while True:
            c, a, m, ln = step(l, rr)
            out.append((rr, l, c, a, m))
            l = ln
            if len(out) >= cap or 1.0 - l <= delta:
                break
        return out, l

    if r > 0:
        out, l = run(r, max_steps)
        return (out, l) if 1.0 - l <= delta else ([], l)
    for rr in range(1, 9):
        out, l = run(rr, 2)
        if 1.0 - l <= delta:
            return out, l
    out, l = run(8, max_steps)
    return (out, l) if 1.0 - l <= delta else ([], l)


def sign_dense(M: np.ndarray, l0: float, delta: float = 1e-15, r: int = 0) -> np.ndarray:
    """Zolo-pd on a small dense matrix M (||M||_2 <= 1, sigma_min >= l0) in FP64: each step
    X <- mhat (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1}), every term in the QR form
    X (X^T X + c I)^{-1} = Q1 Q2^T / sqrt(c) with [X; sqrt(c) I] = [Q1; Q2] R (c_1 is as small as
    l^2, where the normal equations lose everything)."""
    sched, _ = schedule(l0, delta, r)
    X = np.array(M, dtype=np.float64)
    n = X.shape[0]
    for rr, _, c, a, m in sched:
        acc = X.copy()
        for j in range(1, rr + 1):
            sc = math.sqrt(c[2 * j - 1])
            Q, _ = np.linalg.qr(np.vstack([X, sc * np.eye(n)]))
            acc += a[j] / sc * (Q[:n] @ Q[n:].T)
        X = m * acc
    return X

"""Pins of the Zolo-pd oracle (oracle/zolo.py) and the library's coefficients against it."""
import numpy as np
import pytest
from scipy.special import ellipj, ellipk

from oracle import qdwh, zolo


@pytest.mark.parametrize("l", [0.9, 0.5, 0.1, 1e-2, 1e-4, 1e-8, 1e-12, 1e-16])
def test_degree_one_is_the_qdwh_step(l):
    """r = 1: Zhat(x) = mhat x (x^2 + c_2) / (x^2 + c_1) is the QDWH map f(x) = x (a + b x^2) / (1 + c x^2)
    of eq. qdwh_parameters_abc (both are the best type (3, 2) approximation scaled to f(1) = 1)."""
    a, b, c = qdwh.weights(l)
    cz, az, m, ln = zolo.step(l, 1)
    assert abs(cz[1] - 1.0 / c) <= 1e-12 * (1.0 / c)
    assert abs(cz[2] - a / b) <= 1e-12 * (a / b)
    assert abs(m - b / c) <= 1e-12 * (b / c)
    assert abs(ln - float(qdwh.f(l, a, b, c))) <= 1e-12


def _extrema(x, f):
    """Indices of the interior extrema: sign changes of the increments, increments below rounding
    taking the sign of the previous one (flat bottoms do not count twice)."""
    d = np.diff(f)
    s = np.where(np.abs(d) > 1e-13, np.sign(d), 0.0)
    for i in range(1, len(s)):
        if s[i] == 0.0:
            s[i] = s[i - 1]
    idx = np.where(s[1:] * s[:-1] < 0)[0] + 1
    return idx


@pytest.mark.parametrize("l,r", [(0.5, 1), (0.5, 2), (0.1, 3), (1e-3, 4), (1e-8, 4), (1e-16, 6), (1e-16, 8)])
def test_zolotarev_function_equioscillates(l, r):
    """The best approximation equioscillates: on [l, 1] Zhat has r + 1 maxima equal to 1 (x = 1 among
    them) and r + 1 minima equal to Zhat(l) (x = l among them).  A wrong c_i breaks the equality."""
    c, a, m, ln = zolo.step(l, r)
    err = 1.0 - ln
    assert err > 1e-14
    # a grid dense near l, where the extrema of a small l crowd together
    x = np.unique(np.concatenate([np.geomspace(l, 1.0, 400001), np.linspace(l, 1.0, 200001)]))
    f = zolo.zhat(x, c, m, r)
    assert abs(f[-1] - 1.0) <= 1e-14 and abs(f[0] - ln) <= 1e-14
    idx = _extrema(x, f)
    vals = f[idx]
    hi = vals[vals > 1.0 - err / 2]
    lo = vals[vals <= 1.0 - err / 2]
    assert len(hi) == r and len(lo) == r  # interior ones; the endpoints make r + 1 each
    assert np.all(np.abs(hi - 1.0) <= 1e-4 * err + 1e-15)
    assert np.all(np.abs(lo - ln) <= 1e-4 * err + 1e-15)
    assert f.max() <= 1.0 + 1e-4 * err + 1e-15 and f.min() >= ln - 1e-4 * err - 1e-15


@pytest.mark.parametrize("l", [0.9, 0.5, 0.1, 1e-2])
@pytest.mark.parametrize("r", [1, 2, 5, 8])
def test_coefficients_match_scipy_where_representable(l, r):
    """Where m = 1 - l^2 is representable with room to spare, scipy's Jacobi functions give the c_i."""
    m = 1.0 - l * l
    Kp = ellipk(m)
    c, _, _, _ = zolo.step(l, r)
    for i in range(1, 2 * r + 1):
        sn, cn, _, _ = ellipj(i * Kp / (2 * r + 1), m)
        ref = l * l * (sn / cn) ** 2
        assert abs(c[i] - ref) <= 1e-11 * ref, (i, c[i], ref)


@pytest.mark.parametrize("l,r", [(0.5, 3), (1e-5, 5), (1e-16, 8)])
def test_partial_fractions_equal_the_product_form(l, r):
    """a_j are the residues: mhat (x + sum_j a_j x / (x^2 + c_{2j-1})) equals the product form."""
    c, a, m, _ = zolo.step(l, r)
    x = np.geomspace(l, 1.0, 2001)
    pf = m * (x + sum(a[j] * x / (x * x + c[2 * j - 1]) for j in range(1, r + 1)))
    assert np.abs(pf - zolo.zhat(x, c, m, r)).max() <= 1e-13
    assert all(aj > 0 for aj in a[1:])


@pytest.mark.parametrize("l0", [0.5, 1e-3, 1e-8, 1e-16])
def test_two_steps_suffice_and_r_is_minimal(l0):
    sched, lK = zolo.schedule(l0, 1e-15)
    assert len(sched) <= 2 and 1.0 - lK <= 1e-15
    r = sched[0][0]
    if r > 1:  # one degree less does not make it in two steps
        l = l0
        for _ in range(2):
            l = zolo.step(l, r - 1)[3]
        assert 1.0 - l > 1e-15
    if l0 == 1e-16:
        assert r == 8  # the design point of the method (kappa = 1e16, two steps, r = 8)


@pytest.mark.parametrize("lmin,bound", [(1e-4, 1e-11), (1e-9, 1e-6)])
def test_dense_iteration_reaches_the_sign(lmin, bound):
    """The dense iteration against sign(M) from the eigendecomposition: its error is rounding times
    the condition of the sign function (about 1 / lmin), and the scalar map sends every |lambda| to 1."""
    rng = np.random.default_rng(3)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([-np.geomspace(lmin, 1, n // 2), np.geomspace(10 * lmin, 1, n - n // 2)])
    M = (Q * lam) @ Q.T
    M = 0.5 * (M + M.T)
    S = zolo.sign_dense(M, lmin)
    ref = (Q * np.sign(lam)) @ Q.T
    assert np.abs(S - ref).max() <= bound
    sched, _ = zolo.schedule(lmin)
    x = np.abs(lam)
    for rr, _, c, a, m in sched:
        x = m * (x + sum(a[j] * x / (x * x + c[2 * j - 1]) for j in range(1, rr + 1)))
    assert np.abs(x - 1.0).max() <= 4e-15


@pytest.mark.parametrize("l", [0.99, 0.5, 0.1, 1e-3, 1e-6, 1e-10, 1e-16, 1e-40])
@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
def test_library_coefficients_match_the_oracle(l, r):
    """The library's arithmetic-geometric-mean route against the oracle's theta series."""
    import paper_1608_01164_amd as hq
    c, a, m, ln = hq.binding.test_zolo(l, r)
    co, ao, mo, lno = zolo.step(l, r)
    assert np.all(np.abs(c[1:] - np.array(co[1:])) <= 1e-12 * np.array(co[1:]))
    assert np.all(np.abs(a[1:] - np.array(ao[1:])) <= 1e-10 * np.array(ao[1:]))
    assert abs(m - mo) <= 1e-12 * mo
    assert abs(ln - lno) <= 1e-12

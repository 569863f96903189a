"""Pins of the scalar QDWH schedule (CPU only), for the oracle and for the library's host routine.

The weights of eq. qdwh_parameters_abc are defined by an optimality property (Sec. 2.1): among the
maps f(x) = x (a + b x^2) / (1 + c x^2) with b = (a - 1)^2 / 4 and c = a + b - 1 (so 0 < f <= 1 on
(0, 1] and f(1) = 1), a = h(l) is the one that makes the smallest value of f on [l, 1] as large as
possible; l_{k+1} = f_k(l_k) is then that smallest value.  These tests check the property itself
from the critical points of f, not the closed form of h: at the optimum f equioscillates, its
interior local minimum x_m on [l, 1] equals f(l), and moving a either way lowers min over [l, 1]
of f.  A wrong constant anywhere in h moves a off the optimum and fails them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import qdwh

FACTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
LGRID = np.geomspace(1e-16, 0.99, 161)


def f_of(x, a):
    """The rational map of one QDWH step with b and c tied to a as in eq. qdwh_parameters_abc."""
    b = (a - 1.0) ** 2 / 4.0
    c = a + b - 1.0
    x = np.asarray(x, dtype=np.float64)
    return x * (a + b * x * x) / (1.0 + c * x * x)


def critical_points(a):
    """Local maximum x_M and local minimum x_m of f on (0, inf): f'(x) = 0 is the quadratic
    b c y^2 + (3b - a c) y + a = 0 in y = x^2 (numerator of f' = (a + 3 b x^2)(1 + c x^2) - 2 c x^2 (a + b x^2))."""
    b = (a - 1.0) ** 2 / 4.0
    c = a + b - 1.0
    B = a * c - 3.0 * b
    yp = (B + math.sqrt(B * B - 4.0 * a * b * c)) / (2.0 * b * c)
    ym = a / (b * c * yp)  # product of the roots; no cancellation
    return math.sqrt(ym), math.sqrt(yp)


def min_on(l, a):
    """min of f over [l, 1]: f rises to x_M, falls to x_m, rises to f(1) = 1."""
    xM, xm = critical_points(a)
    vals = [float(f_of(l, a)), 1.0]
    if l < xm < 1.0:
        vals.append(float(f_of(xm, a)))
    return min(vals)


def check_optimal(l, a, b, c, rel=1e-12):
    assert abs(b - (a - 1.0) ** 2 / 4.0) <= 1e-15 * b
    assert abs(c - (a + b - 1.0)) <= 1e-15 * c
    xM, xm = critical_points(a)
    assert l < xM < xm < 1.0
    fl, fm = float(f_of(l, a)), float(f_of(xm, a))
    assert abs(fm - fl) <= rel * fl, (l, a, fl, fm)  # equioscillation: the dip equals the value at l
    # the dense-grid minimum over [l, 1] is the value at l
    x = np.concatenate([np.geomspace(l, 1.0, 4001), np.linspace(l, 1.0, 4001)])
    assert f_of(x, a).min() >= fl * (1 - rel)
    # a is the maximiser: both directions lower the minimum
    for d in (1e-6, -1e-6):
        assert min_on(l, a * (1 + d)) < min_on(l, a)


def test_weights_at_one():
    a, b, c = qdwh.weights(1.0)
    assert (a, b, c) == (3.0, 1.0, 3.0)


@pytest.mark.parametrize("l", list(LGRID))
def test_oracle_weights_are_optimal(l):
    a, b, c = qdwh.weights(float(l))
    check_optimal(float(l), a, b, c)
    # the l recurrence is f evaluated at l
    assert abs(float(qdwh.f(l, a, b, c)) - l * (a + b * l * l) / (1 + c * l * l)) <= 1e-15 * l * a


def test_library_schedule_is_optimal():
    """The library's own schedule (host routine behind every solve): every step's weights satisfy the
    optimality property, l_{k+1} = f_k(l_k), and the schedule matches the oracle's."""
    import paper_1608_01164_amd as hq
    for l0 in [1e-16, 1e-12, 3.3e-8, 1.7e-5, 1e-3, 0.2, 0.9]:
        a, b, c, l = hq.binding.test_schedule(l0)
        sched, lK = qdwh.schedule(l0)
        assert len(a) == len(sched) and abs(l[-1] - lK) <= 1e-15
        for k in range(len(a)):
            if l[k] < 0.99:
                check_optimal(l[k], a[k], b[k], c[k])
            assert abs(l[k + 1] - min(1.0, float(f_of(l[k], a[k])))) <= 1e-15
            assert abs(a[k] - sched[k][0]) <= 1e-14 * a[k] and abs(c[k] - sched[k][2]) <= 1e-14 * c[k]


def test_mutated_h_fails_the_pin():
    """The pin is sharp: h with one coefficient changed (8 - 3 g instead of 8 - 4 g) is rejected."""
    def h_bad(l):
        l2 = l * l
        g = (4.0 * (1.0 - l2) / (l2 * l2)) ** (1.0 / 3.0)
        sg = math.sqrt(1.0 + g)
        return sg + 0.5 * math.sqrt(8.0 - 3.0 * g + 8.0 * (2.0 - l2) / (l2 * sg))
    for l in [1e-12, 1e-5, 0.1]:
        a = h_bad(l)
        b = (a - 1) ** 2 / 4
        with pytest.raises(AssertionError):
            check_optimal(l, a, b, a + b - 1)


def test_iteration_bound():
    sched, lK = qdwh.schedule(1e-16, delta=1e-15)
    assert len(sched) <= FACTS["qdwh_max_iterations"]["value"]
    assert abs(1 - lK) <= 1e-15


@pytest.mark.parametrize("l0", [1e-16, 1e-8, 1e-4, 1e-2])
def test_c_decreases_to_three(l0):
    sched, _ = qdwh.schedule(l0)
    cs = [s[2] for s in sched]
    assert all(cs[i] > cs[i + 1] for i in range(len(cs) - 1))
    assert abs(cs[-1] - FACTS["qdwh_c_limit"]["value"]) < 1e-2


def test_map_converges_on_spectrum():
    rng = np.random.default_rng(0)
    l0 = 1e-6
    x = np.concatenate([-np.geomspace(l0, 1, 500), np.geomspace(l0, 1, 500), rng.uniform(-1, 1, 200)])
    x = x[np.abs(x) >= l0]
    sched, _ = qdwh.schedule(l0)
    y = qdwh.iterate_eigenvalues(x, sched)
    assert np.max(np.abs(y - np.sign(x))) < 1e-14

"""Pins of the scalar QDWH schedule (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import qdwh

FACTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_weights_at_one():
    a, b, c = qdwh.weights(1.0)
    assert (a, b, c) == (3.0, 1.0, 3.0)


@pytest.mark.parametrize("l", [1e-16, 1e-10, 1e-5, 1e-3, 0.1, 0.5, 0.9, 0.999])
def test_map_properties(l):
    a, b, c = qdwh.weights(l)
    assert abs(c - (a + b - 1)) < 1e-12 * c
    assert abs(qdwh.f(1.0, a, b, c) - 1.0) < 1e-14
    x = np.linspace(l, 1.0, 20001)
    fx = qdwh.f(x, a, b, c)
    assert np.max(fx) <= 1.0 + 1e-12 and np.max(fx) > 1 - 1e-6
    # the l recurrence is f evaluated at l
    assert abs(qdwh.f(l, a, b, c) - l * (a + b * l * l) / (1 + c * l * l)) < 1e-15


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

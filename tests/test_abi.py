"""The C-ABI library loads and exports every entry point declared in include/hq.h (CPU only)."""
import os
import re

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_]+)\s*\(", src)) - {"if", "while", "for", "sizeof"})


def test_exports_every_declared_symbol():
    import paper_1608_01164_amd as hq
    L = hq.lib()
    names = declared()
    assert "spectral_projector" in names and "apply_projector" in names and "hodlr_build" in names
    for name in names:
        assert hasattr(L, name), name
    # the binding wraps exactly the declared entry points, no more and no fewer
    assert set(names) == set(hq.binding.EXPORTED)


def test_errors_without_device_work():
    import ctypes

    import paper_1608_01164_amd as hq
    L = hq.lib()
    h = ctypes.c_void_p()
    st = L.spectral_projector(None, 10, 1, 2, 0.0, None, None, ctypes.byref(h), None)
    assert st == -1 and h.value is None
    assert b"band" in L.hq_last_error()
    o = hq.Opts()
    assert L.hq_default_opts(ctypes.byref(o)) == 0 and o.leaf == 256 and o.tol == 1e-10
    o.leaf = 1
    st = L.spectral_projector(ctypes.c_void_p(8), 10, 1, 2, 0.0, ctypes.byref(o), None, ctypes.byref(h), None)
    assert st == -1 and b"leaf" in L.hq_last_error()


@pytest.mark.parametrize("maker,b", [(lambda: w.tridiag_uniform(500, 0), 1), (lambda: w.banded_normal(400, 6, 1), 6)])
def test_shift_for_count_matches_oracle(maker, b):
    import paper_1608_01164_amd as hq
    from oracle import eig
    ab = maker()
    n = ab.shape[0]
    mu, gap = hq.shift_for_count(ab, b, n // 2)
    mu_o, gap_o, _ = eig.midpoint_shift(ab, n // 2)
    assert abs(mu - mu_o) < 1e-12 and abs(gap - gap_o) < 1e-12
    assert eig.count(ab, mu) == n // 2


@pytest.mark.parametrize("n,b,leaf", [(2, 1, 2), (16, 1, 4), (100, 4, 12), (257, 5, 40), (600, 1, 64),
                                      (2048, 8, 64)])
def test_structured_qr_host_vs_oracle(n, b, leaf):
    import paper_1608_01164_amd as hq
    from oracle import givens_qr as g
    ab = w.tridiag_uniform(n, 1) if b == 1 else w.banded_normal(n, b, 1)
    A = w.band_to_dense(ab)
    Q, _, rots = g.fast_qr(2.3 * (A - 0.1 * np.eye(n)), b)
    Q1, Q2, nr = hq.test_q_dense_host(ab, b, 0.1, 2.3, leaf)
    assert nr == len(rots) == g.rotation_count(n, b)
    assert np.abs(Q1 - Q[:n, :n]).max() < 1e-13
    assert np.abs(Q2 - Q[n:, :n]).max() < 1e-13
    # the replays run as parallel tasks: the result must not depend on their scheduling
    R1, R2, _ = hq.test_q_dense_host(ab, b, 0.1, 2.3, leaf)
    assert np.array_equal(R1, Q1) and np.array_equal(R2, Q2)


def test_graph_option_is_refused_while_disabled():
    """opts.graph returns HQ_ERR_UNSUPPORTED (checked before any device use)."""
    import ctypes
    import paper_1608_01164_amd as hq
    from paper_1608_01164_amd.binding import _opts
    o = _opts(graph=True)
    out = ctypes.c_void_p()
    st = hq.lib().spectral_projector(ctypes.c_void_p(1), 16, 1, 2, 0.0, ctypes.byref(o), None, ctypes.byref(out), None)
    assert st == -4 and not out.value
    assert b"disabled" in hq.lib().hq_last_error()


def test_tuning_table_is_read_and_checked():
    """The committed autotuner table is what the library uses; out-of-range values are refused."""
    import os
    import paper_1608_01164_amd as hq
    t = hq.tuning()
    path = os.path.join(os.path.dirname(hq.__file__), "tuning.txt")
    assert os.path.samefile(t["source"], path)
    table = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            table[k] = int(v)
    assert all(t[k] == v for k, v in table.items())
    with pytest.raises(hq.HQError):
        hq.set_tuning(qr_tile_rows=8)
    assert hq.tuning()["qr_tile_rows"] == t["qr_tile_rows"]   # a refused table leaves the old one
    old = hq.set_tuning(schur_keep=t["schur_keep"] + 1)
    assert hq.tuning()["schur_keep"] == t["schur_keep"] + 1 and hq.tuning()["source"] == "hq_tuning_set"
    hq.set_tuning(**{k: v for k, v in old.items() if k != "source"})


def test_iteration_records_from_info():
    """Per-iteration log records are built from an info dictionary alone (no library call)."""
    import paper_1608_01164_amd as hq
    info = {"iters": 2, "a": [3.0, 2.5], "b": [1.0, 0.9], "c": [3.5, 3.1], "fp32_iter": [0, 1],
            "max_rank_iter": [12, 15], "iter_seconds": [0.1, 0.2]}
    recs = hq.iteration_records(info, workload="w", step=4)
    assert recs == [
        {"workload": "w", "step": 4, "k": 0, "a": 3.0, "b": 1.0, "c": 3.5, "fp32": False, "max_rank": 12, "seconds": 0.1},
        {"workload": "w", "step": 4, "k": 1, "a": 2.5, "b": 0.9, "c": 3.1, "fp32": True, "max_rank": 15, "seconds": 0.2}]

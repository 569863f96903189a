"""Zolo-pd (opts method='zolo') through the C ABI: the spectral projector against the CPU oracle's
Pi = V V^T, the step schedule against oracle/zolo.py, and the sign function against QDWH's."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w
from oracle import eig, hodlr as oh, norms, zolo

pytestmark = pytest.mark.gpu

GATE = 1e-8  # ||P - Pi_oracle||_2, as for QDWH in FP64


def _dev_band(ab):
    import torch
    return torch.from_numpy(np.ascontiguousarray(ab)).cuda()


CASES = [
    # name, band maker, b, leaf, zolo_r (0: automatic)
    ("dense-leaf", lambda: w.tridiag_uniform(64, 3), 1, 64, 0),
    ("tri-ragged", lambda: w.tridiag_uniform(301, 4), 1, 32, 0),
    ("band3-ragged", lambda: w.banded_normal(257, 3, 5), 3, 32, 0),
    ("metallic", lambda: w.tridiag_metallic(777, 2), 1, 64, 0),
    ("tri-1024-leaf64", lambda: w.tridiag_uniform(1024, 0), 1, 64, 0),
    ("band8-2048-leaf128", lambda: w.banded_normal(2048, 8, 0), 8, 128, 0),
    ("band4-1500-leaf64-r3", lambda: w.banded_normal(1500, 4, 9), 4, 64, 3),
    ("tri-2100-leaf128-r8", lambda: w.tridiag_uniform(2100, 10), 1, 128, 8),
]


@pytest.mark.parametrize("name,maker,b,leaf,r", CASES, ids=[c[0] for c in CASES])
def test_zolo_projector_parity(name, maker, b, leaf, r):
    ab = maker()
    n = ab.shape[0]
    ref = eig.spectral_projector(ab, nu=n // 2)
    P, info = hq.spectral_projector(_dev_band(ab), b, ref.mu, leaf=leaf, tol=1e-10, method="zolo", zolo_r=r)
    H = P.export()
    D = oh.to_dense(H) - ref.Pi
    err2 = norms.lanczos_norm(lambda x: D @ x, n, steps=min(n, 80))
    print(f"{name}: n={n} b={b} gap={ref.gap:.3e} steps={info['iters']} r={info['zolo_r']} "
          f"maxrank={info['max_rank']} redo={info['redo_count']} ||P-Pi||_2={err2:.3e} t={info['seconds']:.3f}s")
    assert err2 <= GATE
    # the steps follow the oracle's schedule for the same l0
    sched, _ = zolo.schedule(info["l0"], 1e-15, r)
    assert len(sched) == info["iters"] and sched[0][0] == info["zolo_r"]
    assert np.allclose([s[4] for s in sched], info["a"], rtol=1e-12)       # mhat_k
    assert np.allclose([s[2][1] for s in sched], info["c"], rtol=1e-12)    # c_1 of each step
    if r == 0:
        assert info["iters"] <= 2


def test_zolo_sign_matches_qdwh():
    """Both methods compute sign(A - mu I); their results agree to the truncation level."""
    ab = w.banded_normal(1800, 3, 11)
    mu, _ = hq.shift_for_count(ab, 3, 900)
    Sz, iz = hq.qdwh_sign(_dev_band(ab), 3, mu, leaf=64, method="zolo")
    Sq, iq = hq.qdwh_sign(_dev_band(ab), 3, mu, leaf=64)
    Dz, Dq = oh.to_dense(Sz.export()), oh.to_dense(Sq.export())
    assert np.linalg.norm(Dz - Dq, 2) <= 1e-8
    assert np.linalg.norm(Dz @ Dz - np.eye(1800), 2) <= 1e-8
    assert iz["iters"] <= 2 < iq["iters"]


def test_zolo_batched_members_equal_single_calls():
    mats = [w.banded_normal(1100, 2, 41), w.tridiag_uniform(900, 42)]
    bws = [2, 1]
    mus = [hq.shift_for_count(m, bw, m.shape[0] // 2)[0] for m, bw in zip(mats, bws)]
    bands = [_dev_band(m) for m in mats]
    Ps, infos, st = hq.spectral_projector_batched(bands, bws, mus, leaf=64, method="zolo")
    assert st == 0
    for j in range(2):
        Pj, _ = hq.spectral_projector(bands[j], bws[j], mus[j], leaf=64, method="zolo")
        assert np.array_equal(oh.to_dense(Pj.export()), oh.to_dense(Ps[j].export()))

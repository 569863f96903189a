"""End-to-end parity: the HIP path's spectral projector against the CPU oracle (FP64)."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w
from tests.mixed_model import bound_from_info
from oracle import eig, hodlr as oh, norms, qdwh

pytestmark = pytest.mark.gpu

GATE = 1e-8  # ||P - Pi_oracle||_2 in FP64 mode


def _dev_band(ab):
    import torch
    return torch.from_numpy(np.ascontiguousarray(ab)).cuda()


CASES = [
    # name, band maker, b, leaf, tol
    ("dense-leaf", lambda: w.tridiag_uniform(64, 3), 1, 64, 1e-10),
    ("tri-ragged", lambda: w.tridiag_uniform(301, 4), 1, 32, 1e-10),
    ("band3-ragged", lambda: w.banded_normal(257, 3, 5), 3, 32, 1e-10),
    ("laplace", lambda: w.laplacian(500), 1, 64, 1e-10),
    ("metallic", lambda: w.tridiag_metallic(777, 2), 1, 64, 1e-10),
    ("tri-1024-leaf64", lambda: w.tridiag_uniform(1024, 0), 1, 64, 1e-10),
    ("band8-2048-leaf128", lambda: w.banded_normal(2048, 8, 0), 8, 128, 1e-10),
    # off-diagonal factors decay to the underflow range (wide gap, 71-row leaves, depth 5)
    ("tri-2284-leaf128-decay", lambda: w.banded_normal(2284, 1, rng=np.random.default_rng([0, 7])), 1, 128, 1e-10),
    # leaves above 128 rows: the leaf Cholesky-inverse splits them 2 x 2 recursively (375 -> 188/187 ->
    # 94/94 ..., 525 -> 263/262 -> 132/131 -> 66/66 ...)
    ("band4-1500-leaf512", lambda: w.banded_normal(1500, 4, 9), 4, 512, 1e-10),
    ("tri-2100-leaf600", lambda: w.tridiag_uniform(2100, 10), 1, 600, 1e-10),
]


@pytest.mark.parametrize("name,maker,b,leaf,tol", CASES, ids=[c[0] for c in CASES])
def test_projector_parity(name, maker, b, leaf, tol):
    ab = maker()
    n = ab.shape[0]
    nu = n // 2
    ref = eig.spectral_projector(ab, nu=nu)
    P, info = hq.spectral_projector(_dev_band(ab), b, ref.mu, leaf=leaf, tol=tol)
    H = P.export()
    D = oh.to_dense(H) - ref.Pi
    err2 = norms.lanczos_norm(lambda x: D @ x, n, steps=min(n, 80))
    print(f"{name}: n={n} b={b} gap={ref.gap:.3e} K={info['iters']} maxrank={info['max_rank']} "
          f"||P-Pi||_2={err2:.3e} t={info['seconds']:.3f}s")
    assert err2 <= GATE
    # schedule agrees with the oracle's scalar recurrence for the same l0
    sched, _ = qdwh.schedule(info["l0"])
    assert len(sched) == info["iters"]
    assert np.allclose([s[2] for s in sched], info["c"], rtol=1e-12)
    # l0 is a certified lower bound of sigma_min((A - mu I)/alpha) within a factor 2
    dist = min(abs(ref.mu - ref.lam[-1]), ref.gap - abs(ref.mu - ref.lam[-1]))
    assert info["l0"] <= dist / info["alpha"] <= 2 * info["l0"] * (1 + 1e-12)
    # apply through the library equals the oracle's matvec on the exported factors
    import torch
    X = np.random.default_rng(0).standard_normal((n, 3))
    Y = P.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(Y - oh.matvec(H, X)).max() < 1e-11
    assert np.abs(Y - ref.apply(X)).max() < 10 * GATE


def test_sign_and_projector_consistent():
    ab = w.tridiag_uniform(400, 9)
    ref = eig.spectral_projector(ab, nu=200)
    S, _ = hq.qdwh_sign(_dev_band(ab), 1, ref.mu, leaf=50)
    P, _ = hq.spectral_projector(_dev_band(ab), 1, ref.mu, leaf=50)
    Sd, Pd = oh.to_dense(S.export()), oh.to_dense(P.export())
    # against the oracle: sign(A - mu I) = I - 2 Pi and Pi itself
    assert np.linalg.norm(Sd - (np.eye(400) - 2.0 * ref.Pi), 2) <= 2 * GATE
    assert np.linalg.norm(Pd - ref.Pi, 2) <= GATE
    # both outputs are truncated independently at tol = 1e-10
    assert np.abs(Pd - 0.5 * (np.eye(400) - Sd)).max() < 1e-9
    assert np.linalg.norm(Sd @ Sd - np.eye(400), 2) < 1e-8


def test_singular_shift_is_reported():
    ab = w.laplacian(64)
    lam = -2 * np.cos(np.pi * 32 / 65)
    with pytest.raises(hq.HQError) as e:
        hq.spectral_projector(_dev_band(ab), 1, lam, leaf=16)
    assert e.value.status == 1


BATCH = [
    # band maker, b (one leaf size for the whole batch)
    (lambda: w.tridiag_uniform(500, 11), 1),
    (lambda: w.banded_normal(257, 3, 12), 3),
    (lambda: w.laplacian(700), 1),
    (lambda: w.tridiag_metallic(777, 13), 1),
    (lambda: w.banded_normal(1024, 8, 14), 8),
    (lambda: w.tridiag_uniform(64, 15), 1),  # a single leaf: dense QDWH
]


def test_batched_parity_and_equal_to_single_calls():
    """Members of uneven size, bandwidth and tree depth advance together; each must meet the
    oracle gate, and equal the single-matrix call bit for bit (the batch only groups launches)."""
    bands, bs, mus, refs = [], [], [], []
    for maker, b in BATCH:
        ab = maker()
        ref = eig.spectral_projector(ab, nu=ab.shape[0] // 2)
        bands.append(_dev_band(ab))
        bs.append(b)
        mus.append(ref.mu)
        refs.append(ref)
    Ps, infos, st = hq.spectral_projector_batched(bands, bs, mus, leaf=64, tol=1e-10)
    assert st == 0
    for i, (P, info, ref) in enumerate(zip(Ps, infos, refs)):
        n = ref.Pi.shape[0]
        Pd = oh.to_dense(P.export())
        err2 = norms.lanczos_norm(lambda x: (Pd - ref.Pi) @ x, n, steps=min(n, 80))
        print(f"member {i}: n={n} b={bs[i]} K={info['iters']} maxrank={info['max_rank']} ||P-Pi||_2={err2:.3e}")
        assert err2 <= GATE
        P1, info1 = hq.spectral_projector(bands[i], bs[i], mus[i], leaf=64, tol=1e-10)
        assert info1["iters"] == info["iters"]
        assert np.array_equal(oh.to_dense(P1.export()), Pd)


def test_batched_reports_failed_member():
    good = w.tridiag_uniform(300, 16)
    ref = eig.spectral_projector(good, nu=150)
    lap = w.laplacian(65)  # 0 is an eigenvalue of the odd-order Laplacian
    Ps, infos, st = hq.spectral_projector_batched([_dev_band(good), _dev_band(lap)], [1, 1], [ref.mu, 0.0], leaf=32)
    assert st == 1 and Ps[1] is None and Ps[0] is not None
    Pd = oh.to_dense(Ps[0].export())
    assert np.linalg.norm(Pd - ref.Pi, 2) <= GATE


MIXED_CASES = [
    ("tri-1024-leaf64", lambda: w.tridiag_uniform(1024, 0), 1, 64),
    ("band8-2048-leaf128", lambda: w.banded_normal(2048, 8, 0), 8, 128),
    ("metallic-777", lambda: w.tridiag_metallic(777, 2), 1, 64),
]
# Stated error level of the mixed mode (tests/mixed_model.py, fixed before the runs): each FP32
# iteration k leaves a perturbation of the size of the FP32 truncation level 4 u32 sqrt(ceil(n/2)) of the
# largest blocks in X_{k+1}; its part that couples eigenvectors across mu turns the invariant subspace by
# about that over 2 l_{k+1}, and the later FP64 iterations do not undo it.
@pytest.mark.parametrize("name,maker,b,leaf", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_precision_projector(name, maker, b, leaf):
    """Mixed mode: middle iterations in FP32.  The error against the oracle is reported and held to
    the stated mixed-mode bound; the FP32 iterations are the ones the schedule allows."""
    ab = maker()
    n = ab.shape[0]
    ref = eig.spectral_projector(ab, nu=n // 2)
    P, info = hq.spectral_projector(_dev_band(ab), b, ref.mu, leaf=leaf, tol=1e-10, precision="mixed")
    D = oh.to_dense(P.export()) - ref.Pi
    err2 = norms.lanczos_norm(lambda x: D @ x, n, steps=min(n, 80))
    K = info["iters"]
    want = [1 if (0 < k < K - 1 and info["c"][k] <= 16.0) else 0 for k in range(K)]
    print(f"mixed {name}: n={n} gap={ref.gap:.3e} K={K} fp32 iterations={info['fp32_iter']} ||P-Pi||_2={err2:.3e}")
    assert info["fp32_iter"] == want and sum(want) >= 1
    bound = bound_from_info(n, info)
    print(f"    stated mixed-mode bound {bound:.2e} ({bound / err2:.1f} x the error)")
    assert err2 <= bound


@pytest.mark.parametrize("n,b,leaf", [(300, 1, 40), (257, 5, 32), (1000, 8, 64)])
def test_hodlr_build_is_exact(n, b, leaf):
    """hodlr_build through the C ABI: X0 = (A - shift I) / scale in HODLR format, every off-diagonal
    block of rank b, equal to the dense matrix up to the rounding of the scaling."""
    ab = w.banded_normal(n, b, 21)
    shift, scale = 0.37, 3.9
    H = hq.hodlr_build(_dev_band(ab), b, shift, scale, leaf=leaf)
    ex = H.export()
    X = oh.to_dense(ex)
    ref = (w.band_to_dense(ab) - shift * np.eye(n)) / scale
    assert np.abs(X - ref).max() <= 4 * np.finfo(float).eps * np.abs(ref).max()
    # every off-diagonal block is stored with rank b (the b x b corner next to the diagonal)
    assert ex["blocks"] and all(F.shape[1] == b for blk in ex["blocks"] for F in blk[3:])
    H.close()


def test_iteration_times_and_records():
    """Each iteration's wall time is reported (positive, summing to at most the call's time) and the
    per-iteration records carry the schedule's weights and the reported ranks."""
    ab = w.banded_normal(1024, 4, 3)
    mu, _ = hq.shift_for_count(ab, 4, 512)
    P, info = hq.spectral_projector(_dev_band(ab), 4, mu, leaf=64, tol=1e-10)
    P.close()
    t = info["iter_seconds"]
    assert len(t) == info["iters"] and all(x > 0 for x in t)
    assert sum(t) <= info["seconds"]
    recs = hq.iteration_records(info, case="band4")
    assert [r["k"] for r in recs] == list(range(info["iters"]))
    assert all(r["case"] == "band4" and r["seconds"] == t[r["k"]] and r["a"] == info["a"][r["k"]] and
               r["max_rank"] == info["max_rank_iter"][r["k"]] for r in recs)

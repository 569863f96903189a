"""Rank predictor: the library's network kernels against the reference network, training, and
what the predictor changes in a solve (capacities) and what it must not change (the result)."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
from paper_1608_01164_amd import predictor as hp
import workloads as w
from oracle import mlp

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _data(rows, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (rows, mlp.F)).astype(np.float32)
    T = rng.uniform(0, 1, (rows, mlp.O)).astype(np.float32)
    W = (rng.uniform(0, 1, (rows, mlp.O)) > 0.25).astype(np.float32)
    return X, T, W


@pytest.mark.parametrize("rows", [1, 127, 128, 1000])
def test_forward_matches_reference(rows):
    import torch
    net = hq.Predictor(seed=rows)
    X, _, _ = _data(rows, rows)
    Y = torch.zeros((rows, mlp.O), dtype=torch.float32, device="cuda")
    net.forward(_t(X), Y)
    ref, _ = mlp.forward(net.params().astype(np.float64), X.astype(np.float64))
    assert np.abs(Y.cpu().numpy() - ref).max() < 2e-5


@pytest.mark.parametrize("rows", [5, 128, 333, 2000])
def test_gradient_matches_reference(rows):
    import torch
    net = hq.Predictor(seed=7)
    rng = np.random.default_rng(rows)
    p = (rng.normal(0, 0.3, net.nparams())).astype(np.float32)
    net.set_params(p)
    X, T, W = _data(rows, rows + 1)
    g = torch.zeros(net.nparams(), dtype=torch.float32, device="cuda")
    loss = net.loss_grad(_t(X), _t(T), _t(W), g)
    L, gref = mlp.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), W.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * max(1.0, L)
    gg = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - gref) <= 1e-4 * np.linalg.norm(gref)
    assert np.abs(gg - gref).max() <= 1e-4 * np.abs(gref).max()


def test_training_fits_a_teacher_network():
    """Targets from another network of the same shape: Adam drives the loss far down."""
    rows = 2048
    X, _, W = _data(rows, 3)
    teacher = np.random.default_rng(4).normal(0, 0.5, mlp.nparams())
    T, _ = mlp.forward(teacher, X.astype(np.float64))
    net = hq.Predictor(seed=5)
    L0 = mlp.loss(net.params().astype(np.float64), X, T, W)
    net.train(_t(X), _t(T.astype(np.float32)), _t(W), epochs=1500, lr=3e-3)
    L1 = mlp.loss(net.params().astype(np.float64), X, T, W)
    assert L1 < 0.02 * L0


def _solve(ab, b, mu, **kw):
    import torch
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    P, info = hq.spectral_projector(band, b, mu, **kw)
    H = P.export()
    P.close()
    return H, info


def _same(H1, H2):
    from oracle import hodlr as oh
    return np.array_equal(oh.to_dense(H1), oh.to_dense(H2))


@pytest.fixture(scope="module")
def small_predictor():
    """Trained in the test on recorded solves of small problems (seeds unlike the checks below)."""
    probs = [(n, b, 300 + i, 64, 1e-10, "band") for i, (n, b) in enumerate(
        [(1024, 1), (1024, 3), (1024, 6), (1500, 2), (1500, 5), (2048, 1), (2048, 4), (2048, 8)])]
    X, T, W = hp.collect(probs)
    net, loss = hp.train(X, T, W, epochs=3000)
    assert loss < 0.01
    return net


@pytest.mark.parametrize("n,b,seed", [(1800, 3, 11), (2048, 6, 12), (1200, 1, 13)])
def test_predictor_keeps_results_and_cuts_capacity(small_predictor, n, b, seed):
    ab = w.banded_normal(n, b, seed)
    mu, _ = hq.shift_for_count(ab, b, n // 2)
    H0, i0 = _solve(ab, b, mu, leaf=64)
    H1, i1 = _solve(ab, b, mu, leaf=64, predictor=small_predictor)
    assert _same(H0, H1)  # capacities never change the arithmetic
    print(f"n={n} b={b}: capacity columns {i0['capacity_columns']} -> {i1['capacity_columns']}, "
          f"peak {i0['peak_bytes'] / 2**20:.1f} -> {i1['peak_bytes'] / 2**20:.1f} MiB, redo {i1['redo_count']}")
    assert i1["capacity_columns"] < 0.85 * i0["capacity_columns"]
    assert i1["peak_bytes"] < i0["peak_bytes"]
    assert i1["redo_count"] <= 1


def test_underpredicting_network_only_costs_redos():
    """A network that predicts rank 0 everywhere: the first Cholesky iteration overflows and is
    repeated with larger capacities; from then on the member's capacities are at least those the
    previous iterate's ranks call for, so few further repeats happen, and the projector is bit for bit
    the one without a predictor."""
    zero = hq.Predictor(seed=0)
    zero.set_params(np.zeros(zero.nparams(), dtype=np.float32))
    ab = w.banded_normal(1500, 4, 21)
    mu, _ = hq.shift_for_count(ab, 4, 750)
    H0, i0 = _solve(ab, 4, mu, leaf=64)
    H1, i1 = _solve(ab, 4, mu, leaf=64, predictor=zero)
    assert 1 <= i1["redo_count"] <= i0["redo_count"] + 2
    assert _same(H0, H1)


def test_recorded_ranks_are_consistent():
    ab = w.banded_normal(2048, 5, 31)
    mu, _ = hq.shift_for_count(ab, 5, 1024)
    import torch
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    P, info = hq.binding._solve("spectral_projector", band, 5, mu, None, raw_info=True, leaf=64, record_ranks=True)
    R = info.level_ranks_array()
    d = info.as_dict()
    assert R.shape == (d["iters"], 4, d["levels"])
    assert list(R[:, 0, :].max(1)) == d["max_rank_iter"]  # X_{k+1} per level vs per iteration
    assert (R[0, 0] <= 3 * 5).all()                      # X_1 has rank <= 3b (structured QR step)
    X, T, Wt = hq.predictor_rows(info, 2048, 5, leaf=64)
    assert len(X) == d["iters"] * d["levels"]
    assert np.allclose(T[:, 0], np.log2(1 + R[:, 0, :].ravel()) / 10, atol=1e-6)
    assert (Wt[: d["levels"], 1:] == 0).all() and (Wt[d["levels"]:] == 1).all()
    P.close()

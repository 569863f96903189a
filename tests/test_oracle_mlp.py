"""Pins of the reference predictor network: finite differences and a closed form."""
import numpy as np

from oracle import mlp


def _data(rows=37, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (rows, mlp.F))
    T = rng.uniform(0, 1, (rows, mlp.O))
    W = (rng.uniform(0, 1, (rows, mlp.O)) > 0.2).astype(np.float64)
    theta = rng.normal(0, 0.4, mlp.nparams())
    return theta, X, T, W


def test_parameter_count_matches_layout():
    assert mlp.nparams() == 32 * 10 + 32 + 32 * 32 + 32 + 4 * 32 + 4 == 1540


def test_gradient_matches_central_differences():
    theta, X, T, W = _data()
    L, g = mlp.loss_grad(theta, X, T, W)
    assert np.isclose(L, mlp.loss(theta, X, T, W), rtol=0, atol=1e-15)
    h = 1e-6
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.nparams(), 200, replace=False), [0, 319, 320, 351, 352, 1407, 1408, 1539]])
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, X, T, W) - mlp.loss(theta - e, X, T, W)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_zero_network_closed_form():
    """All weights and hidden biases zero: y = b3 for every row, so the loss is a weighted mean of
    (b3 - t)^2 and its gradient is 2 sum w (b3 - t) / sum w in b3 and zero elsewhere."""
    _, X, T, W = _data(seed=2)
    theta = np.zeros(mlp.nparams())
    b3 = np.array([0.3, -0.1, 0.7, 0.2])
    theta[-4:] = b3
    L, g = mlp.loss_grad(theta, X, T, W)
    assert np.isclose(L, np.sum(W * (b3 - T) ** 2) / W.sum(), rtol=1e-14)
    assert np.allclose(g[-4:], 2 * np.sum(W * (b3 - T), 0) / W.sum(), rtol=1e-14)
    assert np.all(g[: -36] == 0.0)          # W1, b1, W2, b2: no signal through tanh(0) = 0 with zero W3
    assert np.allclose(g[-36:-4], 0.0)      # W3: h2 = 0


def test_masked_entries_do_not_contribute():
    theta, X, T, W = _data(seed=3)
    T2 = T.copy()
    T2[W == 0] += 100.0
    L1, g1 = mlp.loss_grad(theta, X, T, W)
    L2, g2 = mlp.loss_grad(theta, X, T2, W)
    assert L1 == L2 and np.array_equal(g1, g2)

"""Reference for the rank predictor network (test infrastructure): float64 forward pass, weighted
squared-error loss and its gradient by plain backpropagation, written from the definitions.

Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3, with the flat parameter
vector ordered W1 (H x F, row-major), b1, W2 (H x H), b2, W3 (O x H), b3.
Loss: sum_{i,o} w_io (y_io - t_io)^2 / sum_{i,o} w_io.

Pinned in tests by central finite differences of the loss and by the closed form of the
zero-weight network (y = b3 everywhere).
"""
from __future__ import annotations

import numpy as np

F, H, O = 10, 32, 4


def sizes(f: int = F, h: int = H, o: int = O):
    return [(h, f), (h,), (h, h), (h,), (o, h), (o,)]


def nparams(f: int = F, h: int = H, o: int = O) -> int:
    return sum(int(np.prod(s)) for s in sizes(f, h, o))


def unpack(theta, f: int = F, h: int = H, o: int = O):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for s in sizes(f, h, o):
        k = int(np.prod(s))
        out.append(theta[off: off + k].reshape(s))
        off += k
    assert off == theta.size
    return out


def forward(theta, X, f: int = F, h: int = H, o: int = O):
    """Y (rows x O) and the hidden activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, f, h, o)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3, (h1, h2)


def loss(theta, X, T, W, f: int = F, h: int = H, o: int = O) -> float:
    Y, _ = forward(theta, X, f, h, o)
    W = np.asarray(W, dtype=np.float64)
    return float(np.sum(W * (Y - T) ** 2) / np.sum(W))


def loss_grad(theta, X, T, W, f: int = F, h: int = H, o: int = O):
    """(loss, gradient) by backpropagation through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, f, h, o)
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    Y, (h1, h2) = forward(theta, X, f, h, o)
    ws = np.sum(W)
    E = Y - T
    L = float(np.sum(W * E ** 2) / ws)
    dY = 2.0 * W * E / ws                  # dL/dy
    gW3, gb3 = dY.T @ h2, dY.sum(0)
    dZ2 = (dY @ W3) * (1.0 - h2 ** 2)      # dL/d(pre-activation of layer 2)
    gW2, gb2 = dZ2.T @ h1, dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (1.0 - h1 ** 2)
    gW1, gb1 = dZ1.T @ X, dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g

"""Norm estimates used to compare a result with the oracle -- TEST INFRASTRUCTURE.

lanczos_norm: the 2-norm of a symmetric operator x -> op(x) by the symmetric Lanczos process with
full reorthogonalisation; the largest Ritz value in modulus is a lower bound that is tight after a
few dozen steps for the operators met here.  Pinned by tests/test_oracle_hodlr.py against
numpy.linalg.norm(., 2) on dense symmetric matrices.
"""
from __future__ import annotations

import numpy as np


def lanczos_norm(op, n: int, steps: int = 60, seed: int = 0) -> float:
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(n)
    q /= np.linalg.norm(q)
    Qs = [q]
    alphas, betas = [], []
    beta = 0.0
    q_prev = np.zeros(n)
    for _ in range(min(steps, n)):
        w = op(q)
        a = float(q @ w)
        w = w - a * q - beta * q_prev
        Qm = np.array(Qs).T
        w -= Qm @ (Qm.T @ w)
        w -= Qm @ (Qm.T @ w)
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if beta < 1e-300:
            break
        betas.append(beta)
        q_prev, q = q, w / beta
        Qs.append(q)
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: k - 1], 1) + np.diag(betas[: k - 1], -1)
    return float(np.max(np.abs(np.linalg.eigvalsh(T))))

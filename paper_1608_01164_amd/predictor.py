"""Training and storage of the rank predictor.

Orchestration only: rank traces come from solves recorded by the library (opts record_ranks), the
training rows from the library's feature code (hq_predictor_rows), and the forward/backward/Adam
steps from its kernels.  The default network is trained on seeded synthetic banded problems
(seeds disjoint from the benchmark workloads) and stored as JSON next to this file.

    python -m paper_1608_01164_amd.predictor --train      # on a GPU: rebuild predictor_default.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "predictor_default.json")
FORMAT = "hq-rank-predictor-v1"

# (n, b, seed, leaf, tol, kind): banded N(0,1) (kind "band") or tridiagonal uniform ("tri")
TRAIN_SET = [
    (n, b, 100 + i, 128, 1e-10, "band")
    for i, (n, b) in enumerate([(2048, 1), (2048, 4), (2048, 9), (2048, 16), (3000, 2), (3000, 7), (3000, 13),
                                (4096, 3), (4096, 8), (4096, 12), (4096, 16), (6000, 5), (6000, 10), (6000, 15),
                                (8192, 1), (8192, 6), (8192, 11), (8192, 14), (12000, 4), (12000, 9),
                                (16384, 2), (16384, 8), (16384, 16)])
] + [
    (4096, 1, 140, 256, 1e-10, "tri"), (16384, 1, 141, 256, 1e-10, "tri"), (32768, 1, 142, 256, 1e-8, "tri"),
    (4096, 8, 143, 256, 1e-10, "band"), (2048, 1, 144, 64, 1e-10, "tri"), (4096, 4, 145, 64, 1e-10, "band"),
]


def _workloads():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads
    return workloads


def make_problem(n, b, seed, kind):
    wl = _workloads()
    if kind == "band":
        return wl.banded_normal(n, b, seed)
    if kind == "metallic":  # tridiagonal, diagonal 2 + U(0, 0.1), off-diagonal -1
        return wl.tridiag_metallic(n, seed)
    return wl.tridiag_uniform(n, seed)


def collect(problems, verbose=False):
    """Training rows (X, T, W) from recorded solves of (n, b, seed, leaf, tol, kind) problems."""
    import torch
    Xs, Ts, Ws = [], [], []
    for (n, b, seed, leaf, tol, kind) in problems:
        ab = make_problem(n, b, seed, kind)
        mu, _ = B.shift_for_count(ab, b, n // 2)
        band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
        t0 = time.perf_counter()
        P, info = B._solve("spectral_projector", band, b, mu, None, raw_info=True, leaf=leaf, tol=tol,
                           record_ranks=True)
        P.close()
        X, T, W = B.predictor_rows(info, n, b, leaf=leaf, tol=tol)
        Xs.append(X)
        Ts.append(T)
        Ws.append(W)
        if verbose:
            print(f"# trace n={n} b={b} leaf={leaf} K={info.iters} rows={len(X)} {time.perf_counter() - t0:.2f}s",
                  file=sys.stderr, flush=True)
    return np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ws)


def train(X, T, W, epochs=4000, lr=3e-3, seed=0, quantile=0.995):
    """A new predictor fitted on the rows with the library's Adam kernels; returns (net, loss).

    The capacity margins are set from the residuals: per output, the `quantile` of the amount by
    which the network under-predicts a recorded rank code (at least 0.01), since one
    under-predicted level makes the whole iteration run again."""
    import torch
    net = B.Predictor(seed)
    dX, dT, dW = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in (X, T, W))
    loss = net.train(dX, dT, dW, epochs, lr)
    Y = torch.zeros_like(dT)
    net.forward(dX, Y)
    under = (T - Y.cpu().numpy())
    margin = [max(0.01, float(np.quantile(under[W[:, o] > 0, o], quantile))) if (W[:, o] > 0).any() else 0.05
              for o in range(B.NOUT)]
    net.set_margin(np.minimum(margin, 1.0))
    return net, loss


def save(net, path=DEFAULT_PATH, meta=None):
    doc = {"format": FORMAT, "nparams": net.nparams(), "params": [float(v) for v in net.params()],
           "margin": [float(v) for v in net.margin()], "meta": meta or {}}
    with open(path, "w") as f:
        json.dump(doc, f)


def load(path=DEFAULT_PATH):
    """A predictor with stored parameters (the network lives on the current device)."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != FORMAT:
        raise ValueError(f"{path}: not a rank predictor file")
    net = B.Predictor(0)
    net.set_params(np.asarray(doc["params"], dtype=np.float32))
    net.set_margin(np.asarray(doc["margin"], dtype=np.float32))
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", action="store_true")
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--epochs", type=int, default=4000)
    args = ap.parse_args()
    if not args.train:
        ap.print_help()
        return
    t0 = time.perf_counter()
    X, T, W = collect(TRAIN_SET, verbose=True)
    t1 = time.perf_counter()
    net, loss = train(X, T, W, epochs=args.epochs)
    t2 = time.perf_counter()
    save(net, args.out, {"rows": int(len(X)), "epochs": args.epochs, "loss": loss, "trace_seconds": t1 - t0,
                         "train_seconds": t2 - t1, "problems": [list(p) for p in TRAIN_SET]})
    print(json.dumps({"rows": int(len(X)), "loss": loss, "trace_s": t1 - t0, "train_s": t2 - t1}), flush=True)


if __name__ == "__main__":
    main()

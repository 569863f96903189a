"""Every value the autotuner may choose gives a projector within the parity gate: the tuning table
changes how work is tiled (TSQR row tiles, split-K, when the Schur factor is compressed), never what
is computed.  Each candidate is set for the process, one projector is computed and compared with the
oracle, and the table in use before the test is restored."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w
from oracle import eig, hodlr as oh, norms

pytestmark = pytest.mark.gpu

GATE = 1e-8
CANDIDATES = [
    {"qr_tile_rows": 256}, {"qr_tile_rows": 512}, {"qr_tile_rows": 2048},
    {"split_chunk": 128, "split_min_k": 256}, {"split_chunk": 512, "split_max": 16}, {"split_max": 64},
    {"schur_keep": 0}, {"schur_keep": 160}, {"gemm_small_tiles": 0}, {"gemm_small_tiles": 1 << 20},
]


@pytest.fixture(scope="module")
def problem():
    ab = w.banded_normal(2304, 6, 41)   # 2304 rows: several row tiles at every candidate height
    ref = eig.spectral_projector(ab, nu=2304 // 2)
    return ab, ref


@pytest.mark.parametrize("cand", CANDIDATES, ids=[",".join(f"{k}={v}" for k, v in c.items()) for c in CANDIDATES])
def test_tuning_candidate_parity(problem, cand):
    import torch
    ab, ref = problem
    old = hq.set_tuning(**cand)
    try:
        P, info = hq.spectral_projector(torch.from_numpy(np.ascontiguousarray(ab)).cuda(), 6, ref.mu, leaf=96,
                                        tol=1e-10)
        D = oh.to_dense(P.export()) - ref.Pi
        P.close()
    finally:
        hq.set_tuning(**{k: v for k, v in old.items() if k in cand})
    err = norms.lanczos_norm(lambda x: D @ x, D.shape[0], steps=60)
    print(f"{cand}: ||P - Pi||_2 = {err:.3e}, K={info['iters']}, max rank {info['max_rank']}", flush=True)
    assert err <= GATE

"""HODLR -> H-matrix conversion (hodlr_to_hmatrix, Sec. 3.1.2) through the C ABI: the partition equals
the oracle's (eq. stand_adm), the blocks reassemble the HODLR projector to the truncation level and the
oracle's Pi to the parity gate, and the storage counts match the blocks."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w
from oracle import eig, hmatrix, hodlr as oh, norms

pytestmark = pytest.mark.gpu


def _dev_band(ab):
    import torch
    return torch.from_numpy(np.ascontiguousarray(ab)).cuda()


@pytest.mark.parametrize("name,maker,b,leaf", [
    ("tri-1024-leaf64", lambda: w.tridiag_uniform(1024, 0), 1, 64),
    ("band4-1500-leaf60", lambda: w.banded_normal(1500, 4, 9), 4, 60),
    ("band8-2048-leaf128", lambda: w.banded_normal(2048, 8, 0), 8, 128),
    ("tri-ragged-301-leaf32", lambda: w.tridiag_uniform(301, 4), 1, 32),
])
def test_hmatrix_of_projector(name, maker, b, leaf):
    ab = maker()
    n = ab.shape[0]
    ref = eig.spectral_projector(ab, nu=n // 2)
    P, info = hq.spectral_projector(_dev_band(ab), b, ref.mu, leaf=leaf, tol=1e-10)
    Hh = hq.hodlr_to_hmatrix(P, 1e-10)
    sh = Hh.shape()
    lr, dn = Hh.blocks()
    # the partition is the oracle's, bit for bit
    got = sorted([(r0, c0, U.shape[0], V.shape[0], False) for r0, c0, U, V in lr] +
                 [(r0, c0, D.shape[0], D.shape[1], True) for r0, c0, D in dn])
    assert got == hmatrix.partition(n, leaf)
    # reassembly against the HODLR matrix and against the oracle
    M = np.zeros((n, n))
    for r0, c0, U, V in lr:
        M[r0:r0 + U.shape[0], c0:c0 + V.shape[0]] = U @ V.T
    for r0, c0, D in dn:
        M[r0:r0 + D.shape[0], c0:c0 + D.shape[1]] = D
    Hd = oh.to_dense(P.export())
    # every admissible sub-block is truncated once at 1e-10; a row of blocks holds at most 3 per level
    assert np.linalg.norm(M - Hd, 2) <= 3 * info["levels"] * 1e-10 + 1e-12
    err = norms.lanczos_norm(lambda x: (M - ref.Pi) @ x, n, steps=min(n, 80))
    assert err <= 1e-8
    # storage counts
    nb = sum((U.shape[0] + V.shape[0]) * U.shape[1] for _, _, U, V in lr) + sum(D.size for _, _, D in dn)
    assert sh["bytes"] == 8 * nb and sh["low_rank_blocks"] == len(lr) and sh["dense_blocks"] == len(dn)
    H = P.export()
    hb = sum(l.size for (_, _, l) in H["leaves"]) + sum(
        (U0.shape[0] + V0.shape[0]) * U0.shape[1] + (U1.shape[0] + V1.shape[0]) * U1.shape[1]
        for (_, _, _, U0, V0, U1, V1) in H["blocks"])
    assert sh["hodlr_bytes"] == 8 * hb
    print(f"{name}: n={n} HODLR {sh['hodlr_bytes'] / 2**20:.2f} MB, H {sh['bytes'] / 2**20:.2f} MB "
          f"({sh['low_rank_blocks']} low-rank, {sh['dense_blocks']} dense, max rank {sh['max_rank']}), "
          f"||M - P||_2 {np.linalg.norm(M - Hd, 2):.2e}, ||M - Pi||_2 {err:.2e}")
    assert sh["max_rank"] <= info["max_rank"]
    Hh.close()
    P.close()

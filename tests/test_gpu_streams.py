"""The library issues part of every product and H-Cholesky on side streams (joined through events)
and reuses device and pinned memory across calls.  Races there would show as results that change
from one call to the next; here the same problem is solved repeatedly, alone and inside batches,
and every result must agree bit for bit."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w

pytestmark = pytest.mark.gpu


def _export(P):
    H = P.export()
    P.close()
    return H


def _dense(H):
    from oracle import hodlr as oh
    return oh.to_dense(H)


@pytest.mark.parametrize("n,b,leaf", [(4096, 8, 128), (3000, 3, 64)])
def test_repeated_calls_are_bitwise_identical(n, b, leaf):
    import torch
    ab = w.banded_normal(n, b, 21)
    mu, _ = hq.shift_for_count(ab, b, n // 2)
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    ref = None
    for _ in range(3):
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=1e-10)
        D = _dense(_export(P))
        if ref is None:
            ref = D
        else:
            assert np.array_equal(D, ref)
    # a different problem in between leaves the cached memory with other contents
    ab2 = w.tridiag_uniform(2048, 5)
    mu2, _ = hq.shift_for_count(ab2, 1, 1024)
    P2, _ = hq.spectral_projector(torch.from_numpy(np.ascontiguousarray(ab2)).cuda(), 1, mu2, leaf=64, tol=1e-10)
    P2.close()
    P, _ = hq.spectral_projector(band, b, mu, leaf=leaf, tol=1e-10)
    assert np.array_equal(_dense(_export(P)), ref)


def test_batch_member_equals_single_call():
    """A member solved inside a batch (lockstep launches shared with other members of other tree
    depths) gives the same projector as the same matrix solved alone."""
    import torch
    mats = [w.banded_normal(2500, 4, 31), w.tridiag_uniform(1800, 32), w.banded_normal(1100, 7, 33)]
    bws = [4, 1, 7]
    mus = [hq.shift_for_count(m, bw, m.shape[0] // 2)[0] for m, bw in zip(mats, bws)]
    bands = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
    Ps, infos, st = hq.spectral_projector_batched(bands, bws, mus, leaf=64, tol=1e-10)
    assert st == 0
    for j in range(3):
        Pj, _ = hq.spectral_projector(bands[j], bws[j], mus[j], leaf=64, tol=1e-10)
        Dj = _dense(_export(Pj))
        Db = _dense(_export(Ps[j]))
        # the same arithmetic, only grouped into shared launches: tasks are independent, so the
        # results agree (in practice bit for bit; 1e-12 leaves room for capacity-independent reorderings)
        assert np.abs(Dj - Db).max() <= 1e-12, j


@pytest.mark.skip(reason="opts.graph is disabled: the stream-capture path ended its first GPU run in a host "
                         "segmentation fault whose cause has not been found; the option returns "
                         "HQ_ERR_UNSUPPORTED until it is")
@pytest.mark.parametrize("n,b,leaf", [(4096, 8, 128), (3000, 3, 64)])
def test_graph_iterations_are_bitwise_identical(n, b, leaf):
    """Each Cholesky iteration launched as one captured HIP graph (opts.graph) replays the same
    kernels with the same arguments as the launches issued one by one: the projector is the same bit
    for bit, on repeated calls too."""
    import torch
    ab = w.banded_normal(n, b, 22)
    mu, _ = hq.shift_for_count(ab, b, n // 2)
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=1e-10)
    ref = _dense(_export(P))
    assert info["graphs"] == 0
    for _ in range(2):
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=1e-10, graph=True)
        assert info["graphs"] == info["iters"] - 1 + info["redo_count"] and info["graph_nodes"] > 0
        assert np.array_equal(_dense(_export(P)), ref)

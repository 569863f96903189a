"""Pins of the H-matrix partition oracle (oracle/hmatrix.py), eq. stand_adm of Sec. 3.1.2."""
import numpy as np
import pytest

from oracle import hmatrix


@pytest.mark.parametrize("n,n_min", [(16, 2), (100, 7), (1024, 64), (1000, 60), (16000, 250), (7, 7)])
def test_partition_tiles_the_matrix_and_is_coarsest(n, n_min):
    blocks = hmatrix.partition(n, n_min)
    cover = np.zeros((n, n), dtype=np.int32) if n <= 1024 else None
    nodes, L = hmatrix.cluster_tree(n, n_min)
    leaf_sizes = {hi - lo for lo, hi in nodes[(1 << L) - 1:]}
    area = 0
    for r0, c0, m, k, dense in blocks:
        area += m * k
        if cover is not None:
            cover[r0:r0 + m, c0:c0 + k] += 1
        t, s = (r0, r0 + m), (c0, c0 + k)
        if dense:
            assert not hmatrix.admissible(t, s) and (m in leaf_sizes or k in leaf_sizes)
        else:
            assert hmatrix.admissible(t, s)
    assert area == n * n
    if cover is not None:
        assert (cover == 1).all()  # disjoint and covering
    # coarsest: the cluster pair one level up of every block (its parents) is inadmissible
    parent = {}
    for p in range(1, len(nodes)):
        parent[nodes[p]] = nodes[(p - 1) // 2]
    for r0, c0, m, k, dense in blocks:
        t, s = (r0, r0 + m), (c0, c0 + k)
        if t in parent and s in parent:
            assert not hmatrix.admissible(parent[t], parent[s])


def test_hodlr_block_splits_into_low_rank_blocks_and_one_dense_corner():
    """n = 2^L n_min: the off-diagonal HODLR block of the root (rows a, cols b) holds 3 low-rank blocks
    per level below it and one dense n_min x n_min corner next to the diagonal (at rows a's last leaf,
    columns b's first leaf); every diagonal leaf and its two neighbours are dense."""
    n, n_min, L = 1024, 64, 4
    blocks = hmatrix.partition(n, n_min)
    half = n // 2
    inside = [b for b in blocks if b[0] < half <= b[1]]  # rows in a = [0, n/2), cols in b = [n/2, n)
    lr = [b for b in inside if not b[4]]
    dn = [b for b in inside if b[4]]
    assert len(lr) == 3 * (L - 1) and len(dn) == 1
    assert dn[0][:4] == (half - n_min, half, n_min, n_min)
    dense = {(b[0], b[1]) for b in blocks if b[4]}
    for i in range(0, n, n_min):
        assert (i, i) in dense
        if i + n_min < n:
            assert (i, i + n_min) in dense and (i + n_min, i) in dense
    assert not any(b[4] and abs(b[0] - b[1]) > n_min for b in blocks)


def test_admissibility_definition_on_small_intervals():
    # diam = size - 1, dist = gap + 1 between the nearest indices
    assert hmatrix.admissible((0, 4), (8, 12))        # diam 3 <= dist 5
    assert hmatrix.admissible((0, 4), (7, 11))        # 3 <= 4
    assert not hmatrix.admissible((0, 4), (4, 8))     # 3 > 1 (adjacent)
    assert hmatrix.admissible((0, 2), (2, 4))         # diam 1 <= dist 1
    assert not hmatrix.admissible((0, 4), (2, 6))     # overlapping: dist 0

"""H-matrix block partition with the standard admissibility condition -- TEST INFRASTRUCTURE.

Sec. 3.1.2 (eq. stand_adm): the index set I = {0, ..., n-1} is bisected recursively as for HODLR
(the same cluster tree: [lo, hi) split at lo + ceil((hi - lo) / 2), leaves of at most n_min
indices, all at one depth); a block t x s of two clusters on one level is admissible iff
    min(diam t, diam s) <= dist(t, s),   diam t = max |i - j| over t,  dist(t, s) = min |i - j|, i in t, j in s,
and the recursion over the children pairs stops at an admissible block (stored in low rank) or when
t or s is a leaf cluster (stored dense).

Pinned by (tests/test_oracle_hmatrix.py): the blocks tile I x I exactly; every low-rank block is
admissible and every dense one has a leaf cluster; the parent pair of every block was inadmissible
(the partition is the coarsest one); the diagonal and the blocks next to it are dense, while a
HODLR off-diagonal block splits into low-rank blocks and one dense corner next to the diagonal.
"""
from __future__ import annotations


def cluster_tree(n: int, n_min: int):
    """Nodes (lo, hi) in heap order (children of p: 2p+1, 2p+2) and the depth L."""
    L = 0
    while -(-n // (1 << L)) > n_min:
        L += 1
    nodes = [(0, n)]
    for l in range(L):
        for p in range((1 << l) - 1, (1 << (l + 1)) - 1):
            lo, hi = nodes[p]
            mid = lo + -(-(hi - lo) // 2)
            nodes.append((lo, mid))
            nodes.append((mid, hi))
    return nodes, L


def admissible(t, s) -> bool:
    (a0, a1), (b0, b1) = t, s
    diam = min(a1 - a0 - 1, b1 - b0 - 1)
    if a1 <= b0:
        dist = b0 - a1 + 1
    elif b1 <= a0:
        dist = a0 - b1 + 1
    else:
        dist = 0
    return diam <= dist


def partition(n: int, n_min: int):
    """Sorted list of (row0, col0, rows, cols, dense) blocks."""
    nodes, L = cluster_tree(n, n_min)
    first_leaf = (1 << L) - 1
    out = []

    def rec(p, q):
        t, s = nodes[p], nodes[q]
        if t[1] - t[0] <= 0 or s[1] - s[0] <= 0:
            return
        if admissible(t, s):
            out.append((t[0], s[0], t[1] - t[0], s[1] - s[0], False))
        elif p >= first_leaf or q >= first_leaf:
            out.append((t[0], s[0], t[1] - t[0], s[1] - s[0], True))
        else:
            for pc in (2 * p + 1, 2 * p + 2):
                for qc in (2 * q + 1, 2 * q + 2):
                    rec(pc, qc)

    rec(0, 0)
    return sorted(out)


def storage_doubles(blocks, ranks):
    """Doubles to store the blocks: (rows + cols) * rank for low-rank blocks, rows * cols for dense."""
    tot = 0
    for (r0, c0, m, k, dense) in blocks:
        tot += m * k if dense else (m + k) * ranks[(r0, c0)]
    return tot

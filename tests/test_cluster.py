"""The clustered block partition (Section 6.1; eq. (extended_set) of Section
6.1.1): the oracle's breadth-first block growing pinned by a hand-worked
example and by properties the definition fixes, and the library's host
implementation (sic_cluster_order) equal to it bit for bit. No GPU."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.cluster import adjacency, cluster_order, neighbourhood_sizes
from synth import generators as g


def _keys(P):
    C = sp.triu(sp.csr_matrix(P), k=1).tocoo()
    return (C.row.astype(np.int64) * P.shape[0] + C.col).astype(np.int64)


def test_hand_worked_order():
    # path 0-3-5-1-6 and the edge 2-4, blocks of 3. Degrees 1,2,1,2,1,2,1, so the
    # least-degree order is 0,2,4,6,1,3,5.
    #   block 1: seed 0 (no candidates, least degree); 0 -> 3; 3 -> 5: full.
    #            candidates: the unplaced neighbours of 0, 3, 5: [1]
    #   block 2: seed 1; 1 -> 6 (5 is placed); exhausted with 2 of 3; no
    #            candidates, so the least-degree unplaced vertex 2 joins: full.
    #            candidates: neighbours of 1, 6, 2: [4]
    #   block 3: seed 4 (one vertex left)
    n = 7
    keys = [0 * n + 3, 3 * n + 5, 1 * n + 5, 1 * n + 6, 2 * n + 4, 3 * n + 3]
    assert list(cluster_order(n, keys, 3)) == [0, 3, 5, 1, 6, 2, 4]


def _relabelled_grid(rows, cols, seed):
    rng = np.random.default_rng(seed)
    n = rows * cols
    lab = rng.permutation(n)
    keys = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            for w in ([v + 1] if c + 1 < cols else []) + ([v + cols] if r + 1 < rows else []):
                a, b = sorted((int(lab[v]), int(lab[w])))
                keys.append(a * n + b)
    return n, np.asarray(keys, dtype=np.int64)


def _connected(adj, verts):
    verts = set(verts)
    start = next(iter(verts))
    seen, stack = {start}, [start]
    while stack:
        u = stack.pop()
        for w in adj[u]:
            if w in verts and w not in seen:
                seen.add(w)
                stack.append(w)
    return seen == verts


@pytest.mark.parametrize("b", [16, 64, 100])
def test_blocks_partition_and_stay_connected_on_a_grid(b):
    n, keys = _relabelled_grid(24, 30, seed=b)
    order = cluster_order(n, keys, b)
    assert sorted(order.tolist()) == list(range(n))            # a permutation
    adj = adjacency(n, keys)
    blocks = [order[j0:j0 + b] for j0 in range(0, n, b)]
    # most blocks are one connected piece (those grown from leftovers may not be)
    connected = sum(_connected(adj, blk) for blk in blocks)
    assert connected >= 0.8 * len(blocks)
    # and the neighbourhoods are far smaller than those of the random labels
    nat = np.mean(neighbourhood_sizes(n, keys, np.arange(n), b))
    clu = np.mean(neighbourhood_sizes(n, keys, order, b))
    assert clu < 0.3 * nat


def test_isolated_vertices_and_components():
    # two triangles, an edge and isolated vertices: every vertex placed once,
    # each triangle kept whole in blocks of 3
    n = 12
    keys = [0 * n + 5, 5 * n + 9, 0 * n + 9, 2 * n + 7, 7 * n + 11, 2 * n + 11, 3 * n + 4]
    order = cluster_order(n, keys, 3).tolist()
    assert sorted(order) == list(range(n))
    blocks = [set(order[j:j + 3]) for j in range(0, n, 3)]
    assert {0, 5, 9} in blocks and {2, 7, 11} in blocks


def test_library_order_equals_the_oracle():
    """sic_cluster_order is host code of the library: no device work."""
    from paper_1607_00315_amd import sic
    cases = []
    n, keys = _relabelled_grid(20, 25, seed=3)
    cases.append((n, keys, 64))
    rng = np.random.default_rng(4)
    R = g.random_precision(800, 2400, rng)
    cases.append((800, _keys(R), 50))
    D = g.delaunay_precision(900, np.random.default_rng(5))
    cases.append((D.shape[0], _keys(D), 64))
    # repeated and diagonal keys, isolated vertices
    k = np.concatenate([_keys(R)[:300], _keys(R)[:100], np.arange(0, 800 * 800, 801)])
    cases.append((800, k, 32))
    for n, keys, b in cases:
        assert np.array_equal(sic.cluster_order(n, keys, b), cluster_order(n, keys, b)), (n, b)

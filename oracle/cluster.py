"""Oracle (test infrastructure only): the clustered block partition.

Section 6.1 (and Section 6.1.1, eq. (extended_set)) leaves the partition of
the variables into blocks free and asks for one that keeps the neighbourhoods
N_j small: the paper partitions the graph of the free set (with METIS, which
is not available here) so that each block's free pairs mostly stay inside it.
This reading grows the blocks greedily on that graph, in the spirit of the
graph-growing heuristics of multilevel partitioners:

  * the graph: vertices 0..n-1, an edge for every free pair (i, j), i != j;
  * blocks of exactly b vertices (the last one shorter), formed one after
    another; the order of the variables is the blocks' vertices in order, so
    that the contiguous blocks of the relabelled problem are the clusters;
  * a block grows breadth-first from a seed over vertices not yet placed,
    visiting each vertex's neighbours in ascending order, until it holds b
    vertices; when the growth runs out (its component is exhausted) it goes
    on from the next seed;
  * the next seed is the oldest not yet placed vertex among the candidates
    (vertices adjacent to an earlier block, queued when that block was
    completed, block members in order and each one's neighbours ascending),
    and when there is none, the not yet placed vertex of least degree (ties:
    smaller index).

Plain Python loops: for the small graphs of the tests.
"""

from __future__ import annotations

from collections import deque

import numpy as np


def adjacency(n: int, keys) -> list[list[int]]:
    """Sorted neighbour lists of the graph of pair keys i*n + j (diagonal
    keys and duplicates are ignored)."""
    nb = [set() for _ in range(n)]
    for key in keys:
        i, j = divmod(int(key), n)
        if i != j:
            nb[i].add(j)
            nb[j].add(i)
    return [sorted(s) for s in nb]


def cluster_order(n: int, keys, b: int) -> np.ndarray:
    """Order of the variables whose consecutive runs of b are the blocks."""
    adj = adjacency(n, keys)
    by_degree = sorted(range(n), key=lambda v: (len(adj[v]), v))
    placed = [False] * n
    cand = deque()
    order = []
    sp = 0
    while len(order) < n:
        need = min(b, n - len(order))
        block = []
        while len(block) < need:
            seed = None
            while cand:
                v = cand.popleft()
                if not placed[v]:
                    seed = v
                    break
            if seed is None:
                while placed[by_degree[sp]]:
                    sp += 1
                seed = by_degree[sp]
            placed[seed] = True
            block.append(seed)
            queue = deque([seed])
            while queue and len(block) < need:
                u = queue.popleft()
                for w in adj[u]:
                    if len(block) == need:
                        break
                    if not placed[w]:
                        placed[w] = True
                        block.append(w)
                        queue.append(w)
        for u in block:
            for w in adj[u]:
                if not placed[w]:
                    cand.append(w)
        order.extend(block)
    return np.asarray(order, dtype=np.int64)


def neighbourhood_sizes(n: int, keys, order, b: int) -> list[int]:
    """|N_j| of each block of the relabelled problem: the vertices outside the
    block joined to it by a pair (eq. (extended_set), read as in steps.py)."""
    adj = adjacency(n, keys)
    order = list(order)
    sizes = []
    for j0 in range(0, n, b):
        blk = set(order[j0:j0 + b])
        nbrs = set()
        for u in blk:
            nbrs.update(w for w in adj[u] if w not in blk)
        sizes.append(len(nbrs))
    return sizes

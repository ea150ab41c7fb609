"""Exhaustive optimal partitions for tiny graphs (the problem is NP-complete,
Section 3.2, so the exact optimum is only reachable by enumeration).

Capacity-feasible: at most k = ceil(m/cap) parts, each of at most cap edges.
Set partitions are enumerated as restricted-growth strings.
"""

from __future__ import annotations

import math

import numpy as np

from .cost import partition_cost, weighted_cost
from .graph import clone_and_connect, vertex_cut


def restricted_growth(m: int, max_blocks: int, cap: int):
    """Every assignment a[0..m-1] with a[0] = 0, a[i] <= 1 + max(a[:i]),
    at most max_blocks distinct blocks and at most cap items per block."""
    a = [0] * m
    sizes = [0] * max_blocks

    def rec(i, nb):
        if i == m:
            yield list(a)
            return
        for b in range(min(nb + 1, max_blocks)):
            if sizes[b] < cap:
                a[i] = b
                sizes[b] += 1
                yield from rec(i + 1, max(nb, b + 1))
                sizes[b] -= 1

    if m == 0:
        yield []
        return
    yield from rec(0, 0)


def min_edge_partition_cost(edges, n: int, cap: int, w=None):
    """Minimum C (or, with vertex weights w, sum_v w[v] (p_v - 1)) over all capacity-feasible
    edge partitions, and one minimiser."""
    m = len(edges)
    k = math.ceil(m / cap)
    best, arg = None, None
    for a in restricted_growth(m, k, cap):
        c = partition_cost(edges, n, a, k)["cost"] if w is None else weighted_cost(edges, n, a, w)
        if best is None or c < best:
            best, arg = c, a
    return best, np.asarray(arg)


def min_vertex_partition_cut(edges, n: int, cap: int):
    """Optimal capacity-feasible vertex partition of the contracted index-order
    transform: minimum number of cut auxiliary edges, and one minimiser
    (returned as an edge partition, i.e. already reconstructed)."""
    m = len(edges)
    k = math.ceil(m / cap)
    dp = clone_and_connect(np.asarray(edges), n)
    best, arg = None, None
    for a in restricted_growth(m, k, cap):
        clone_part = np.repeat(np.asarray(a), 2)
        c = vertex_cut(dp, clone_part)
        if best is None or c < best:
            best, arg = c, a
    return best, np.asarray(arg)

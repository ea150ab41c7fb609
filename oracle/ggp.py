"""Balanced edge partition through the transformed graph (Section 3.2).

Steps, in the paper's order:
 1. clone-and-connect (Definition 3), clones chained in ascending edge id;
 2. original edges get "a very large weight" so the vertex partition never cuts
    them; read here as contracting each original edge into one node, which is
    the infinite-weight limit;
 3. balanced vertex partition of the transformed graph; the paper runs METIS,
    which is absent, so this reading uses greedy graph growing (below);
 4. reconstruction (Definition 4), the identity on contracted nodes.

Balance reading: Eq. 1 asks for exactly m/k edges per cluster while the paper
accepts a balance factor near 1.03; here a hard capacity ``cap`` with
k = ceil(m/cap), parts 0..k-2 filled to exactly cap and the last to the rest.

Greedy graph growing, part p = 0..k-1 in turn, one node at a time:
  g[e] = number of links from e to nodes already placed in part p,
  t[e] = number of links from e to nodes already placed in any part;
  pick the unplaced node with the largest g > 0 (ties: smallest id);
  if none has g > 0, the unplaced node with the largest t > 0 (ties: smallest id);
  otherwise the smallest unplaced id.
Links count with multiplicity (parallel edges adjacent in both chains count
twice).  The order of placement is the task order inside each part.

Under input order, part[e] = e // cap and the task order is the identity.
"""

from __future__ import annotations

import heapq
import math

import numpy as np

from .graph import contracted_links, incidence


def partition(edges: np.ndarray, n: int, cap: int, order: str = "ep"):
    """Return (part[m], task_order[m]) as int64 arrays."""
    edges = np.asarray(edges, dtype=np.int64)
    m = len(edges)
    if cap < 1:
        raise ValueError("capacity must be >= 1")
    if order == "input":
        return np.arange(m) // cap, np.arange(m)
    if order != "ep":
        raise ValueError(order)
    k = math.ceil(m / cap) if m else 0
    nbr = contracted_links(edges, n, incidence(edges, n))
    part = [-1] * m
    t = [0] * m
    t_heap = []  # entries (-t, e); stale when e is placed or t[e] moved on
    task = []
    smallest = 0
    for p in range(k):
        size = min(cap, m - p * cap)
        g = {}
        g_heap = []
        for _ in range(size):
            e = _pop_best(g_heap, g, part)
            if e is None:
                e = _pop_best(t_heap, t, part)
            if e is None:
                while part[smallest] != -1:
                    smallest += 1
                e = smallest
            part[e] = p
            task.append(e)
            for f in nbr[e]:
                if part[f] == -1:
                    g[f] = g.get(f, 0) + 1
                    heapq.heappush(g_heap, (-g[f], f))
                    t[f] += 1
                    heapq.heappush(t_heap, (-t[f], f))
    return np.asarray(part, dtype=np.int64), np.asarray(task, dtype=np.int64)


def _pop_best(heap, val, part):
    """Unplaced node with the largest positive value, smallest id on ties."""
    while heap:
        negv, e = heap[0]
        cur = val[e] if isinstance(val, list) else val.get(e, 0)
        if part[e] == -1 and cur == -negv and cur > 0:
            heapq.heappop(heap)
            return e
        heapq.heappop(heap)
    return None

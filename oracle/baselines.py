"""Edge-partition baselines the paper compares against (Section 3.3): the
vertex-cut placements of PowerGraph (Gonzalez et al., OSDI 2012), random and
greedy, under the same hard capacity as the other orders: k = ceil(m/cap)
parts of at most cap edges.

Random: edges sorted by the SplitMix64 hash of their id (ties by id), then
consecutive blocks of cap.  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):
z = x + golden-ratio increment, then two xor-shift-multiply rounds and a final
xor-shift, all mod 2^64.

Greedy, edges in ascending id.  A(v) = parts already holding an edge of v,
rem(v) = edges of v not yet placed, candidates = parts holding fewer than cap
edges, "least loaded" = fewest edges, then smaller id:
  A(u), A(v) share a part      -> least loaded candidate among the shared parts;
  both non-empty, none shared  -> least loaded candidate of A(w), w the endpoint
                                  with more unplaced edges (ties: u);
  one endpoint placed          -> least loaded candidate of its A;
  otherwise, or no candidate   -> least loaded candidate overall.
Tasks inside a part run in ascending edge id.

Greedy is pinned exactly on a hand-derived 9-edge case
(tests/golden/greedy_vertex_cut9.json) that takes each of the four cases
above, on a 5-edge case where the endpoints tie (greedy_tie5.json), and by
capacity, balance and closed forms in the tests; random by SplitMix64's
published outputs.  On larger graphs the exact placement has no value
independent of these rules; there the library is compared with the oracle bit
for bit.
"""

from __future__ import annotations

import math

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def random_partition(m: int, cap: int):
    order = sorted(range(m), key=lambda e: (splitmix64(e), e))
    task = np.array(order, dtype=np.int64)
    part = np.empty(m, dtype=np.int64)
    part[task] = np.arange(m) // cap
    return part, task


def greedy_partition(edges, n: int, cap: int):
    edges = np.asarray(edges, dtype=np.int64)
    m = len(edges)
    k = math.ceil(m / cap) if m else 0
    load = [0] * k
    rem = [0] * n
    for u, v in edges.tolist():
        rem[u] += 1
        rem[v] += 1
    A = [set() for _ in range(n)]

    def least(cands):
        best = None
        for p in sorted(cands):
            if load[p] < cap and (best is None or load[p] < load[best]):
                best = p
        return best

    part = np.empty(m, dtype=np.int64)
    for e, (u, v) in enumerate(edges.tolist()):
        p = None
        if A[u] and A[v]:
            shared = A[u] & A[v]
            if shared:
                p = least(shared)
            else:
                p = least(A[v] if rem[v] > rem[u] else A[u])
        elif A[u]:
            p = least(A[u])
        elif A[v]:
            p = least(A[v])
        if p is None:
            p = least(range(k))
        part[e] = p
        load[p] += 1
        A[u].add(p)
        A[v].add(p)
        rem[u] -= 1
        rem[v] -= 1
    task = np.array(sorted(range(m), key=lambda e: (part[e], e)), dtype=np.int64)
    return part, task

"""The hub split before the EP partition: an extension of the paper's
partition step (Section 3.2) for graphs with a power-law degree distribution,
where the multilevel heuristic scatters the edges of a high-degree vertex over
far more parts than its degree needs.  Not in the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition, stated plainly:
* degree = number of incident edges (multi-edges counted);
* an edge's key is its class-y endpoint (ids at or above n_x; every vertex
  when n_x = 0); of two such endpoints, the one of larger degree, ties to the
  smaller id;
* an edge is a hub edge when it has a key of degree above hub_degree;
* the hub edges, sorted by (key, the other endpoint, edge id), fill parts
  0, 1, ... in runs of cap;
* the remaining edges, in ascending edge id, are partitioned on their own by
  the EP order (``multilevel.partition``, with the class weights), and their
  parts follow the hub parts;
* the task order lists the hub parts' edges in sorted order, then the
  remaining edges in the EP order's task order.

Pins: a hand-derived case (``tests/golden/hub_split7.json``), the reduction to
the plain EP order when no vertex exceeds hub_degree, and invariants (every
edge once, capacity, a hub of degree d in at most ceil(d/cap) + 1 parts)."""

import numpy as np

from . import multilevel


def _key(u, v, deg, n_x):
    yu, yv = u >= n_x, v >= n_x
    if yu and yv:
        return u if (deg[u] > deg[v] or (deg[u] == deg[v] and u < v)) else v
    if yu:
        return u
    if yv:
        return v
    return None


def partition(edges, n, cap, hub_degree, class_weight=None, n_x=0):
    """(part[m], task[m], k) of the hub split followed by the EP order on the rest."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    m = len(E)
    deg = np.zeros(n, dtype=np.int64)
    for u, v in E:
        deg[u] += 1
        deg[v] += 1
    hub, rest = [], []
    for e in range(m):
        u, v = int(E[e, 0]), int(E[e, 1])
        h = _key(u, v, deg, n_x)
        if h is not None and deg[h] > hub_degree:
            hub.append((h, v if h == u else u, e))
        else:
            rest.append(e)
    hub.sort()
    part = np.zeros(m, dtype=np.int64)
    task = []
    for j, (_, _, e) in enumerate(hub):
        part[e] = j // cap
        task.append(e)
    kh = -(-len(hub) // cap)
    k = kh
    if rest:
        p_r, t_r, k_r = multilevel.partition(E[rest], n, cap, class_weight, n_x)
        for j, e in enumerate(rest):
            part[e] = kh + p_r[j]
        task.extend(rest[t] for t in t_r)
        k = kh + k_r
    return part, np.asarray(task, dtype=np.int64), k

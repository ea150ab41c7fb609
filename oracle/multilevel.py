"""Multilevel balanced partition of the contracted transform (Section 3.2).

The paper partitions the clone-and-connect graph D' with METIS, a multilevel
vertex partitioner with a small balance tolerance (its balance factor is
"typically < 1.03").  METIS is absent; this is this project's own multilevel
scheme written from the published method (coarsen by heavy-edge matching,
partition the coarsest graph, project back and refine the boundary), applied
to D' with original edges contracted (infinite weight, so never cut):

* node = an edge of the data-affinity graph, weight 1;
* link weight = number of auxiliary edges of D' between two contracted nodes
  (with per-class vertex weights, the sum of the weights of the vertices whose
  chains those auxiliary edges link: the cost becomes sum_v w(v) (p_v - 1),
  Definition 2 with weighted copies, and Theorem 1 holds for it with the
  weighted cut).

Capacity reading: a hard maximum of c edges per part with 5% room,
k = ceil(m / (c - floor(c/20))) parts, growth target T = ceil(m / k), so the
balance factor max / mean stays <= c / (c - floor(c/20)) (1.05 at c = 256).

1. Coarsen while the graph has more than 16k nodes: visit nodes in ascending
   id; an unmatched node u joins the unmatched neighbour v != u of largest link
   weight (ties: smallest id) with w(u) + w(v) <= W; else it stays single.
   W = min(max(2, floor(c/32)), floor(c/20) + 1): a coarse node weighs at most
   one more than the room the capacity leaves above the growth target, so a
   part below the target always has room for the next node and growing fills
   every part to the target (with no room, c < 20, W = 1 and nothing merges).
   Coarse ids follow the visiting order; weights and link weights add; links
   inside a coarse node vanish.  A level that keeps more
   than 90% of the nodes is discarded and coarsening stops.
2. Partition the coarsest graph by greedy growing (parts 0..k-1 in turn, as in
   ``ggp`` but with node weights: a candidate must fit under c; candidates that
   do not fit are dropped from the queues), place any remainder on a part with
   room (by the weight rule above there is none), then refine, make parts
   contiguous, refine.
3. Project level by level to the finest graph; refine; make parts contiguous.

Inside a part, tasks run in ascending edge id.
"""

from __future__ import annotations

import heapq
import math

import numpy as np

from .graph import contracted_links, incidence


def max_node_weight(cap: int) -> int:
    """Largest coarse-node weight: at most the room (floor(cap/20)) plus one.

    Growth fills part p while its size is below the target T <= cap - floor(cap/20);
    a node of weight w <= floor(cap/20) + 1 then always fits (size + w <= T - 1 + w
    <= cap), so every part reaches T and k*T >= m places every node.
    """
    return min(max(2, cap // 32), cap // 20 + 1)


def parameters(m: int, cap: int):
    """(k, growth target, maximum coarse-node weight)."""
    if m == 0:
        return 0, 0, max_node_weight(cap)
    k = math.ceil(m / (cap - cap // 20))
    return k, math.ceil(m / k), max_node_weight(cap)


def _finest(edges, n, class_weight=None, n_x=0):
    """Contracted D': node e per edge, a link weight per pair of nodes.  Each auxiliary edge
    (consecutive edges of vertex v's incidence list) adds the weight of v's class (x: v < n_x,
    y: the rest) to its link, 1 without class weights."""
    m = len(edges)
    adj = [dict() for _ in range(m)]
    if class_weight is None:
        nbr = contracted_links(edges, n, incidence(edges, n))
        for e in range(m):
            for f in nbr[e]:
                adj[e][f] = adj[e].get(f, 0) + 1
        return adj, [1] * m
    inc = incidence(edges, n)
    for v in range(n):
        w = class_weight[0] if v < n_x else class_weight[1]
        chain = inc[v]
        for t in range(len(chain) - 1):
            a, b = chain[t], chain[t + 1]
            adj[a][b] = adj[a].get(b, 0) + w
            adj[b][a] = adj[b].get(a, 0) + w
    return adj, [1] * m


def coarsen(adj, w, maxw):
    n = len(adj)
    match = [-1] * n
    cmap = [-1] * n
    nc = 0
    for u in range(n):
        if match[u] >= 0:
            continue
        best, bw = -1, 0
        for v, lw in adj[u].items():
            if v != u and match[v] < 0 and w[u] + w[v] <= maxw and (lw > bw or (lw == bw and v < best)):
                best, bw = v, lw
        match[u] = best if best >= 0 else u
        cmap[u] = nc
        if best >= 0:
            match[best] = u
            cmap[best] = nc
        nc += 1
    cw = [0] * nc
    cadj = [dict() for _ in range(nc)]
    for u in range(n):
        cu = cmap[u]
        cw[cu] += w[u]
        for v, lw in adj[u].items():
            cv = cmap[v]
            if cv != cu:
                cadj[cu][cv] = cadj[cu].get(cv, 0) + lw
    return cadj, cw, cmap


def _pop_fitting(heap, val, part, room):
    """Best valid entry that fits in the current part; stale or oversized entries are dropped."""
    while heap:
        negv, x = heapq.heappop(heap)
        if part[x] == -1 and val.get(x, 0) == -negv and room(x):
            return x
    return None


def grow(adj, w, k, target, cap):
    n = len(adj)
    part = [-1] * n
    t = {}
    t_heap = []
    smallest = 0
    placed = 0
    for p in range(k):
        if placed == n:
            break
        size = 0
        g = {}
        g_heap = []
        while size < target:
            def fits(x):
                return size + w[x] <= cap

            e = _pop_fitting(g_heap, g, part, fits)
            if e is None:
                e = _pop_fitting(t_heap, t, part, fits)
            if e is None:
                while smallest < n and part[smallest] != -1:
                    smallest += 1
                if smallest >= n or not fits(smallest):
                    break
                e = smallest
            part[e] = p
            size += w[e]
            placed += 1
            for f, lw in adj[e].items():
                if part[f] == -1:
                    g[f] = g.get(f, 0) + lw
                    heapq.heappush(g_heap, (-g[f], f))
                    t[f] = t.get(f, 0) + lw
                    heapq.heappush(t_heap, (-t[f], f))
    sizes = [0] * k
    for u in range(n):
        if part[u] >= 0:
            sizes[part[u]] += w[u]
    for u in range(n):
        if part[u] == -1:
            conn = {}
            for v, lw in adj[u].items():
                if part[v] >= 0 and sizes[part[v]] + w[u] <= cap:
                    conn[part[v]] = conn.get(part[v], 0) + lw
            if conn:
                p = max(conn, key=lambda q: (conn[q], -q))
            else:
                room = [q for q in range(k) if sizes[q] + w[u] <= cap]
                if not room:
                    raise RuntimeError("no part has room for a remaining node")
                p = min(room, key=lambda q: (sizes[q], q))
            part[u] = p
            sizes[p] += w[u]
    return part


def refine(adj, w, part, k, cap, passes=8):
    n = len(adj)
    sizes = [0] * k
    for u in range(n):
        sizes[part[u]] += w[u]
    for _ in range(passes):
        moved = 0
        for u in range(n):
            a = part[u]
            conn = {}
            for v, lw in adj[u].items():
                conn[part[v]] = conn.get(part[v], 0) + lw
            own = conn.get(a, 0)
            best, bg = -1, 0
            for b, c in conn.items():
                if b == a:
                    continue
                gain = c - own
                if gain > 0 and (gain > bg or (gain == bg and b < best)) and sizes[b] + w[u] <= cap \
                        and sizes[a] - w[u] >= 1:
                    best, bg = b, gain
            if best >= 0:
                part[u] = best
                sizes[a] -= w[u]
                sizes[best] += w[u]
                moved += 1
        if moved == 0:
            break
    return part


def contiguity(adj, w, part, k, cap):
    """Pieces of every part are found first (links inside the part); then, part
    by part in ascending id, every piece but the heaviest (ties: smallest
    member id) moves, heaviest first, to the adjacent part with most link
    weight from it (ties: smallest id) if that part has room."""
    n = len(adj)
    sizes = [0] * k
    for u in range(n):
        sizes[part[u]] += w[u]
    seen = [False] * n
    pieces = [[] for _ in range(k)]
    for u in range(n):
        if seen[u]:
            continue
        seen[u] = True
        stack, mem = [u], [u]
        while stack:
            x = stack.pop()
            for v in adj[x]:
                if not seen[v] and part[v] == part[u]:
                    seen[v] = True
                    stack.append(v)
                    mem.append(v)
        pieces[part[u]].append(mem)
    for p in range(k):
        ps = pieces[p]
        if len(ps) <= 1:
            continue
        ps = sorted(ps, key=lambda mem: (-sum(w[x] for x in mem), min(mem)))
        for mem in ps[1:]:
            wt = sum(w[x] for x in mem)
            conn = {}
            for x in mem:
                for v, lw in adj[x].items():
                    if part[v] != p:
                        conn[part[v]] = conn.get(part[v], 0) + lw
            cand = [q for q in conn if sizes[q] + wt <= cap]
            if not cand:
                continue
            q = max(cand, key=lambda q: (conn[q], -q))
            for x in mem:
                part[x] = q
            sizes[p] -= wt
            sizes[q] += wt
    return part


def partition(edges: np.ndarray, n: int, cap: int, class_weight=None, n_x: int = 0):
    """Return (part[m], task_order[m], k) as int64 arrays / int.  class_weight = (x, y):
    per-class vertex weights of the weighted cost sum_v w(v) (p_v - 1), x being v < n_x."""
    edges = np.asarray(edges, dtype=np.int64)
    m = len(edges)
    if cap < 1:
        raise ValueError("capacity must be >= 1")
    k, target, maxw = parameters(m, cap)
    if m == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), 0
    adj, w = _finest(edges, n, class_weight, n_x)
    levels = []
    while len(adj) > 16 * k:
        cadj, cw, cmap = coarsen(adj, w, maxw)
        if 10 * len(cadj) > 9 * len(adj):
            break
        levels.append((adj, w, cmap))
        adj, w = cadj, cw
    part = grow(adj, w, k, target, cap)
    part = refine(adj, w, part, k, cap)
    part = contiguity(adj, w, part, k, cap)
    part = refine(adj, w, part, k, cap)
    for fadj, fw, cmap in reversed(levels):
        part = [part[cmap[u]] for u in range(len(fadj))]
        part = refine(fadj, fw, part, k, cap)
        part = contiguity(fadj, fw, part, k, cap)
    part = np.asarray(part, dtype=np.int64)
    task = np.lexsort((np.arange(m), part))  # parts ascending, edge id inside a part
    return part, task, k

"""Partition cost: Definition 2 and Eq. 1 written out.

For an edge partition part[e] in [0, k):
  V(P_i) = { u_e, v_e : part[e] = i }      vertices part i must load
  p_v    = #{ i : v in V(P_i) }             clusters that touch v
  L      = sum_i |V(P_i)|                   distinct-vertex loads
  C      = sum over active v of (p_v - 1)   redundant loads (data reuse cost)
  R      = #{ v : p_v >= 2 }                replicated vertices
  S      = sum over p_v >= 2 of p_v         (part, vertex) pairs of replicated vertices
Reading: the sum defining C runs over active vertices (degree >= 1) only; the
literal sum over all of V would give -1 per isolated vertex.  Hence
C = L - n_active and S = C + R.
Balance: max part size / mean part size (Section 3.2), mean = m / k.
aux_cut: the number of auxiliary edges of the index-order transform whose two
endpoint edges lie in different parts.
"""

from __future__ import annotations

import numpy as np


def partition_cost(edges: np.ndarray, n: int, part, k: int | None = None) -> dict:
    edges = np.asarray(edges, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    m = len(edges)
    if k is None:
        k = int(part.max()) + 1 if m else 0
    # distinct (part, vertex) pairs: the loads
    pv_part = np.concatenate([part, part])
    pv_vert = np.concatenate([edges[:, 0], edges[:, 1]])
    pairs = np.unique(pv_part * n + pv_vert) if m else np.zeros(0, dtype=np.int64)
    L = int(len(pairs))
    p_v = np.bincount(pairs % n, minlength=n) if m else np.zeros(n, dtype=np.int64)
    active = p_v >= 1
    n_active = int(active.sum())
    C = int((p_v[active] - 1).sum())
    R = int((p_v >= 2).sum())
    S = int(p_v[p_v >= 2].sum())
    sizes = np.bincount(part, minlength=k) if m else np.zeros(k, dtype=np.int64)
    verts_per_part = np.bincount(pairs // n, minlength=k) if m else np.zeros(k, dtype=np.int64)
    balance = float(sizes.max() / (m / k)) if m and k else 0.0
    return {
        "n_parts": int(k),
        "loads": L,
        "cost": C,
        "replicated": R,
        "slots": S,
        "n_active": n_active,
        "aux_cut": aux_cut(edges, part),
        "max_part_edges": int(sizes.max()) if k else 0,
        "max_part_vertices": int(verts_per_part.max()) if k else 0,
        "balance": balance,
        "p_v": p_v,
    }


def aux_cut(edges: np.ndarray, part) -> int:
    """Cut auxiliary edges of the index-order clone-and-connect transform."""
    edges = np.asarray(edges, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    m = len(edges)
    if m == 0:
        return 0
    vert = np.concatenate([edges[:, 0], edges[:, 1]])
    eid = np.concatenate([np.arange(m), np.arange(m)])
    srt = np.lexsort((eid, vert))
    vert, eid = vert[srt], eid[srt]
    link = vert[1:] == vert[:-1]  # consecutive entries of one vertex's chain
    a, b = eid[:-1][link], eid[1:][link]
    return int((part[a] != part[b]).sum())


def loads_simple(edges, part) -> int:
    """L by sets, for small graphs: sum over parts of the number of distinct vertices."""
    groups = {}
    for (u, v), p in zip(np.asarray(edges).tolist(), np.asarray(part).tolist()):
        groups.setdefault(p, set()).update((u, v))
    return sum(len(s) for s in groups.values())


def weighted_cost(edges: np.ndarray, n: int, part, w) -> int:
    """Definition 2's cost with vertex weights: sum over active v of w[v] (p_v - 1).
    w[v] = 1 for every v is C itself."""
    p_v = partition_cost(edges, n, part)["p_v"]
    w = np.asarray(w, dtype=np.int64)
    active = p_v >= 1
    return int((w[active] * (p_v[active] - 1)).sum())


def weighted_aux_cut(edges: np.ndarray, part, w) -> int:
    """Cut auxiliary edges of the index-order transform, each weighing w of the vertex whose
    chain it links (Theorem 1 with weights: weighted_cost <= weighted_aux_cut)."""
    edges = np.asarray(edges, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    m = len(edges)
    if m == 0:
        return 0
    vert = np.concatenate([edges[:, 0], edges[:, 1]])
    eid = np.concatenate([np.arange(m), np.arange(m)])
    srt = np.lexsort((eid, vert))
    vert, eid = vert[srt], eid[srt]
    link = vert[1:] == vert[:-1]
    a, b, v = eid[:-1][link], eid[1:][link], vert[:-1][link]
    return int((w[v] * (part[a] != part[b])).sum())

"""Data-affinity graph and the clone-and-connect transform.

Definition 1: a vertex per data object, an edge per task using two objects.
Definition 3: every vertex of degree d becomes d clones, one per incident edge;
the clones of a vertex are joined into a path by d-1 auxiliary edges; every
original edge joins the two clones that belong to it.  The clones of a vertex
are chained "in index order" (Section 3.2), read here as ascending edge id.
Definition 4: a vertex partition of the transformed graph that cuts no original
edge maps back to an edge partition: an edge goes where its two clones are.
"""

from __future__ import annotations

import numpy as np


def incidence(edges: np.ndarray, n: int) -> list:
    """inc[v] = ascending list of the ids of the edges incident to v."""
    inc = [[] for _ in range(n)]
    for e, (u, v) in enumerate(np.asarray(edges).tolist()):
        inc[u].append(e)
        inc[v].append(e)
    return inc


def clone_and_connect(edges: np.ndarray, n: int, inc: list | None = None) -> dict:
    """Explicit transformed graph D' of Definition 3.

    Clone ids: the clone of u_e on edge e is 2e, the clone of v_e is 2e + 1.
    Returns the 2m clones' owners, the m original edges (2e, 2e+1) and the
    auxiliary edges that chain each vertex's clones in ascending edge id.
    """
    edges = np.asarray(edges)
    m = len(edges)
    if inc is None:
        inc = incidence(edges, n)
    owner = np.empty(2 * m, dtype=np.int64)
    owner[0::2] = edges[:, 0]
    owner[1::2] = edges[:, 1]

    def clone(v, e):
        return 2 * e if edges[e, 0] == v else 2 * e + 1

    original = [(2 * e, 2 * e + 1) for e in range(m)]
    aux = []
    for v in range(n):
        chain = inc[v]
        for t in range(len(chain) - 1):
            aux.append((clone(v, chain[t]), clone(v, chain[t + 1])))
    return {"n_clones": 2 * m, "owner": owner, "original": original, "aux": aux}


def contracted_links(edges: np.ndarray, n: int, inc: list | None = None) -> list:
    """D' with every original edge contracted to one node (infinite weight).

    Node e stands for both clones of edge e.  nbr[e] lists, with multiplicity,
    the predecessor and successor of e in inc[u_e] and in inc[v_e]: these are
    exactly the auxiliary edges of D' incident to e's two clones.
    """
    edges = np.asarray(edges)
    m = len(edges)
    if inc is None:
        inc = incidence(edges, n)
    nbr = [[] for _ in range(m)]
    for v in range(n):
        chain = inc[v]
        for t in range(len(chain) - 1):
            a, b = chain[t], chain[t + 1]
            nbr[a].append(b)
            nbr[b].append(a)
    return nbr


def reconstruct(dprime: dict, clone_part) -> np.ndarray:
    """Definition 4: edge e goes to the part holding both of its clones."""
    clone_part = np.asarray(clone_part)
    m = len(dprime["original"])
    part = np.empty(m, dtype=np.int64)
    for e, (a, b) in enumerate(dprime["original"]):
        if clone_part[a] != clone_part[b]:
            raise ValueError(f"original edge {e} is cut")
        part[e] = clone_part[a]
    return part


def vertex_cut(dprime: dict, clone_part) -> int:
    """Edge-cut cost of a vertex partition of D': the number of cut auxiliary edges."""
    clone_part = np.asarray(clone_part)
    return int(sum(1 for a, b in dprime["aux"] if clone_part[a] != clone_part[b]))


def rechain_by_part(edges: np.ndarray, n: int, part) -> dict:
    """The transform used in the proof of Theorem 2, for a given edge partition.

    Each vertex's clones are grouped by the part of their edge, chained within
    each group, and the groups chained together (groups in ascending part id,
    clones in ascending edge id inside a group).
    """
    edges = np.asarray(edges)
    part = np.asarray(part)
    inc = incidence(edges, n)
    regrouped = [sorted(chain, key=lambda e: (int(part[e]), e)) for chain in inc]
    return clone_and_connect(edges, n, inc=regrouped)

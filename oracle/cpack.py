"""Data layout along the task order (Section 4.1, cpack).

The paper reorganises the data array along the new task schedule with
Ding and Kennedy's cpack and passes the kernel a remapped index array.  cpack
places data consecutively in the order the task sequence first accesses them;
the reading here is exactly that:

* walk the tasks part by part (ascending part id) and, inside a part, in task
  order, taking u then v of every edge; each vertex takes the next packed id of
  its class at its first touch.  The vertices first touched in part p (the ones
  p OWNS) therefore form one contiguous range per part and class, in
  first-touch order;
* vertices never touched (isolated) follow, in ascending original id;
* SpMV graphs have two classes, x (original id < n_x) and y; each is packed on
  its own, x into [0, n_x) and y into [n_x, n).

The vertices part p uses, per class, are listed as: the ones it owns (first
touched in p, a contiguous packed range) in packed order, then the foreign ones
(owned by an earlier part) in ascending packed id.
"""

from __future__ import annotations

import numpy as np


def layout(edges: np.ndarray, n: int, part, task, n_x: int | None = None) -> dict:
    edges = np.asarray(edges, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    task = np.asarray(task, dtype=np.int64)
    m = len(edges)
    k = int(part.max()) + 1 if m else 0
    bipartite = n_x is not None
    base = [0, n_x] if bipartite else [0]

    def cls(w):
        return 1 if (bipartite and w >= n_x) else 0

    # the order of first touches along the task sequence, and the part of each
    first_touch = []
    first_part = np.full(n, -1, dtype=np.int64)
    prev = -1
    for e in task.tolist():
        p = int(part[e])
        if p < prev:
            raise ValueError("task order must visit parts in ascending id")
        prev = p
        for w in (int(edges[e, 0]), int(edges[e, 1])):
            if first_part[w] < 0:
                first_part[w] = p
                first_touch.append(w)

    nxt = list(base)
    o2p = np.full(n, -1, dtype=np.int64)
    own_start = np.zeros((k, len(base)), dtype=np.int64)  # class counters when part p begins
    i = 0
    for p in range(k):
        own_start[p] = nxt
        while i < len(first_touch) and first_part[first_touch[i]] == p:
            w = first_touch[i]
            c = cls(w)
            o2p[w] = nxt[c]
            nxt[c] += 1
            i += 1
    for w in range(n):
        if o2p[w] < 0:
            c = cls(w)
            o2p[w] = nxt[c]
            nxt[c] += 1
    perm = np.empty(n, dtype=np.int64)
    perm[o2p] = np.arange(n)

    parts = []
    ncls = len(base)
    touched = [[set() for _ in range(ncls)] for _ in range(k)]
    for e in range(m):
        p = int(part[e])
        for w in (int(edges[e, 0]), int(edges[e, 1])):
            touched[p][cls(w)].add(w)
    for p in range(k):
        info = {"own0": [], "nown": [], "foreign": []}
        for c in range(ncls):
            owned = sorted(o2p[w] for w in touched[p][c] if first_part[w] == p)
            foreign = sorted(o2p[w] for w in touched[p][c] if first_part[w] != p)
            if owned and owned != list(range(owned[0], owned[0] + len(owned))):
                raise AssertionError("owned vertices of a part must be contiguous")
            if owned and owned[0] != own_start[p, c]:
                raise AssertionError("owned range must start at the class counter")
            info["own0"].append(int(own_start[p, c]))
            info["nown"].append(len(owned))
            info["foreign"].append(np.asarray(foreign, dtype=np.int64))
        parts.append(info)
    return {"perm": perm, "orig_to_packed": o2p, "parts": parts, "first_part": first_part}


def local_ids(layout_: dict, edges: np.ndarray, part, task) -> list:
    """Per part, the (local u, local v) index pairs in task order.

    The local index of a vertex is its position in the part's vertex list
    (owned then foreign); for two classes the y list follows the x list.
    """
    edges = np.asarray(edges, dtype=np.int64)
    o2p = layout_["orig_to_packed"]
    out = []
    per_part_tasks = {}
    for e in np.asarray(task).tolist():
        per_part_tasks.setdefault(int(part[e]), []).append(e)
    for p, info in enumerate(layout_["parts"]):
        pos = {}
        off = 0
        for c in range(len(info["own0"])):
            ulist = list(range(info["own0"][c], info["own0"][c] + info["nown"][c])) + info["foreign"][c].tolist()
            for i, w in enumerate(ulist):
                pos[w] = off + i
            off += len(ulist)
        pairs = [(pos[o2p[edges[e, 0]]], pos[o2p[edges[e, 1]]]) for e in per_part_tasks.get(p, [])]
        out.append(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    return out

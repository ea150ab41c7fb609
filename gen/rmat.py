"""R-MAT power-law bipartite graphs (SpMV-style workloads).

The paper's SpMV data-affinity graph has one vertex per element of x and of y
and one edge (x_j, y_i) per nonzero A[i, j] (Section 5.2).  Its power-law inputs
(in-2004, scircuit) are absent, so an R-MAT matrix with the recursive quadrant
probabilities (a, b, c, d) stands in for them.  No noise is added, ids are not
permuted and duplicate (i, j) pairs are kept as distinct tasks.
"""

from __future__ import annotations

import numpy as np

from .meshes import _rng

_TAG_RMAT = 11
_TAG_W = 12
_TAG_X = 13
_TAG_SHUF = 14


def rmat(scale: int = 20, n_edges: int = 1 << 24, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 0) -> dict:
    """R-MAT with 2^scale rows and columns.

    Per edge and per level one uniform draw picks a quadrant: [0,a) top-left,
    [a,a+b) top-right (column bit set), [a+b,a+b+c) bottom-left (row bit set),
    else bottom-right (both).  Level 0 sets the most significant bit.

    Returns rows i, cols j (int32), weights w ~ U[0,1) (float32) and x ~ N(0,1)
    (float32, length 2^scale), edges in generation order, plus ``shuffle``:
    a seeded permutation giving the default (shuffled) task order.
    """
    N = 1 << scale
    rng = _rng(seed, _TAG_RMAT)
    row = np.zeros(n_edges, dtype=np.int64)
    col = np.zeros(n_edges, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lev in range(scale):
        r = rng.random(n_edges, dtype=np.float64)
        bit = np.int64(1) << np.int64(scale - 1 - lev)
        colbit = ((r >= a) & (r < ab)) | (r >= abc)
        rowbit = r >= ab
        col |= colbit.astype(np.int64) * bit
        row |= rowbit.astype(np.int64) * bit
        del r
    w = _rng(seed, _TAG_W).random(n_edges, dtype=np.float32)
    x = _rng(seed, _TAG_X).standard_normal(N, dtype=np.float32)
    shuffle = _rng(seed, _TAG_SHUF).permutation(n_edges)
    return {
        "kind": "rmat",
        "n_x": N,
        "n_y": N,
        "rows": row.astype(np.int32),
        "cols": col.astype(np.int32),
        "w": w,
        "x": x,
        "shuffle": shuffle,
    }


def spmv_graph(R: dict, order: np.ndarray | None = None) -> dict:
    """Bipartite data-affinity graph of an R-MAT matrix: edge (j, n_x + i)."""
    rows, cols, w = R["rows"], R["cols"], R["w"]
    if order is not None:
        rows, cols, w = rows[order], cols[order], w[order]
    n_x = R["n_x"]
    edges = np.stack([cols.astype(np.int64), n_x + rows.astype(np.int64)], axis=1).astype(np.int32)
    return {"n": n_x + R["n_y"], "n_x": n_x, "edges": edges, "w": np.ascontiguousarray(w)}

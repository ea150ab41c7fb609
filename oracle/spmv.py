"""SpMV over the bipartite data-affinity graph (Section 5.2).

One vertex per element of x and of y; each nonzero A[i, j] is an edge between
x_j and y_i and the task computes y_i += w_e x_j.  Graph ids: x_j is j and
y_i is n_x + i.  Duplicate (i, j) pairs are distinct tasks and add up.
"""

from __future__ import annotations

import numpy as np


def forward(n_x: int, n_y: int, edges: np.ndarray, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    edges = np.asarray(edges, dtype=np.int64)
    j = edges[:, 0]
    i = edges[:, 1] - n_x
    return np.bincount(i, weights=np.asarray(w, np.float64) * np.asarray(x, np.float64)[j], minlength=n_y)


def forward_abs(n_x: int, n_y: int, edges: np.ndarray, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    edges = np.asarray(edges, dtype=np.int64)
    j = edges[:, 0]
    i = edges[:, 1] - n_x
    return np.bincount(i, weights=np.abs(np.asarray(w, np.float64)) * np.abs(np.asarray(x, np.float64))[j],
                       minlength=n_y)


def row(n_x: int, edges: np.ndarray, w: np.ndarray, x: np.ndarray, i: int):
    """y_i and its absolute-value evaluation for one row, from the edges of that row."""
    edges = np.asarray(edges, dtype=np.int64)
    sel = edges[:, 1] == n_x + i
    t = np.asarray(w, np.float64)[sel] * np.asarray(x, np.float64)[edges[sel, 0]]
    return float(t.sum()), float(np.abs(t).sum())


def backward(n_x: int, n_y: int, edges: np.ndarray, w: np.ndarray, x: np.ndarray, g_y: np.ndarray):
    """Adjoint of y = A x: g_x = A^T g_y (g_x[j] = sum over edges (j, i) of w g_y[i]) and the
    weight gradient g_w[e] = g_y[i] x[j], both in FP64."""
    edges = np.asarray(edges, dtype=np.int64)
    j = edges[:, 0]
    i = edges[:, 1] - n_x
    w64 = np.asarray(w, np.float64)
    gy = np.asarray(g_y, np.float64)
    g_x = np.bincount(j, weights=w64 * gy[i], minlength=n_x)
    g_w = gy[i] * np.asarray(x, np.float64)[j]
    return g_x, g_w


def backward_abs(n_x: int, n_y: int, edges: np.ndarray, w: np.ndarray, x: np.ndarray, g_y: np.ndarray):
    """The same sums over absolute values (the rounding-error scale of each output)."""
    return backward(n_x, n_y, edges, np.abs(np.asarray(w, np.float64)), np.abs(np.asarray(x, np.float64)),
                    np.abs(np.asarray(g_y, np.float64)))

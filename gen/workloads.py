"""Named synthetic workloads and vertex states.

Five workloads mirror the five benchmark configurations:

* ``grid64``   : 2D triangulated 64x64 lattice, n = 4096, m = 12,033, capacity 256.
* ``tet32``    : 3D Kuhn 32^3 dual, n = 196,608, m = 387,072, capacity 256.
* ``rmat20``   : R-MAT 2^20 x 2^20 with 2^24 nonzeros, SpMV, capacity 256.
* ``batch256`` : 256 mesh graphs, vertex counts log-uniform in [1024, 65536].
* ``tet55``    : 3D Kuhn 55^3 dual, n = 998,250, m = 1,978,350, forward + adjoint.

Vertex states are 5 float32 components (density, three momenta, energy) drawn
from U[0.5, 1.5], stored row-major [n][5].
"""

from __future__ import annotations

import math

import numpy as np

from .meshes import _rng, grid2d, tet_mesh
from .rmat import rmat

_TAG_STATE = 21
_TAG_BATCH = 22
_TAG_GRAD = 23

WORKLOADS = {
    "grid64": dict(kind="flux", builder="grid2d", args=(64, 64), cap=256),
    "tet32": dict(kind="flux", builder="tet_mesh", args=(32, 32, 32), cap=256),
    "rmat20": dict(kind="spmv", builder="rmat", args=(20, 1 << 24), cap=256),
    "batch256": dict(kind="batch", builder="batch_graphs", args=(256,), cap=None),
    "tet55": dict(kind="flux", builder="tet_mesh", args=(55, 55, 55), cap=256),
    # a mesh whose step working set (~0.45 GB) exceeds the 256 MiB MALL: back-to-back steps stream HBM
    "tet80": dict(kind="flux", builder="tet_mesh", args=(80, 80, 80), cap=256),
}


def flux_state(n: int, seed: int = 0, tag: int = _TAG_STATE) -> np.ndarray:
    """Vertex states q[n][5] ~ U[0.5, 1.5], float32."""
    return _rng(seed, tag).uniform(0.5, 1.5, size=(n, 5)).astype(np.float32)


def grad_seed(n: int, seed: int = 0) -> np.ndarray:
    """Upstream gradient g_r[n][5] ~ N(0, 1), float32 (for adjoint parity)."""
    return _rng(seed, _TAG_GRAD).standard_normal(size=(n, 5)).astype(np.float32)


def workload(name: str, seed: int = 0) -> dict:
    spec = WORKLOADS[name]
    if spec["builder"] == "grid2d":
        g = grid2d(*spec["args"], seed=seed)
    elif spec["builder"] == "tet_mesh":
        g = tet_mesh(*spec["args"], seed=seed)
    elif spec["builder"] == "rmat":
        g = rmat(*spec["args"], seed=seed)
    else:
        g = {"graphs": batch_graphs(*spec["args"], seed=seed)}
    g["cap"] = spec["cap"]
    g["name"] = name
    return g


def batch_graphs(n_graphs: int = 256, seed: int = 0, lo: int = 1024, hi: int = 65536) -> list:
    """Uneven batch: graph g has N_g = round(exp(U(ln lo, ln hi))) target vertices.

    Even g: 2D lattice with W = ceil(sqrt(N)), H = round(N / W).
    Odd g : Kuhn a x a x c box, a = max(2, round((N/6)^(1/3))), c = max(1, round(N / (6 a^2))).
    Every graph carries 4 geometry floats per edge (2D graphs: (nx, ny, 0, 1)).
    """
    rng = _rng(seed, _TAG_BATCH)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_graphs))).astype(np.int64)
    out = []
    for gi, N in enumerate(sizes):
        if gi % 2 == 0:
            W = int(math.ceil(math.sqrt(N)))
            H = max(2, int(round(N / W)))
            g = grid2d(W, H, seed=seed * 100003 + gi)
            geom = np.concatenate([g["geom"], np.zeros((len(g["edges"]), 1)), np.ones((len(g["edges"]), 1))], axis=1)
            g["geom"] = geom
        else:
            a = max(2, int(round((N / 6.0) ** (1.0 / 3.0))))
            c = max(1, int(round(N / (6.0 * a * a))))
            g = tet_mesh(a, a, c, seed=seed * 100003 + gi)
        g["target_n"] = int(N)
        out.append(g)
    return out

"""Seeded synthetic inputs shaped like the paper's workloads.

This package builds graphs, geometry and vertex states only. It holds none of
the method's arithmetic (no partitioning, no packing, no flux), so that both the
FP64 oracle and the HIP path can draw the same inputs from it without sharing
any code of the method.

Every random quantity comes from its own PCG64 stream seeded with
``SeedSequence([seed, tag])``, so adding a draw never shifts another one.
"""

from .meshes import grid2d, tet_mesh, bfs_subgraph, default_order
from .rmat import rmat
from .workloads import (
    flux_state,
    WORKLOADS,
    workload,
    batch_graphs,
)

__all__ = [
    "grid2d",
    "tet_mesh",
    "bfs_subgraph",
    "default_order",
    "rmat",
    "flux_state",
    "WORKLOADS",
    "workload",
    "batch_graphs",
]

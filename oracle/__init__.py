"""FP64 CPU oracle for the edge-partitioned kernel path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library and imports nothing
from it; the two meet only in the seeded input generators (package ``gen``).

Each function is a plain, slow, obviously-correct statement of what the method
computes, written from the paper (arXiv 1605.02043, "A Graph-based Model for
GPU Caching Problems"):

* ``graph``   - data-affinity graph, clone-and-connect transform, reconstruction
                (Definitions 1, 3, 4).
* ``cost``    - partition cost C, loads L and friends (Definition 2, Eq. 1).
* ``multilevel`` - the balanced vertex partition of the transformed graph
                (Section 3.2; the paper uses METIS, which is absent), read as a
                deterministic multilevel partitioner: the EP order.
* ``ggp``     - the same step read as single-pass greedy graph growing.
* ``cpack``   - first-touch data packing along the task order (Section 4.1).
* ``flux``    - the cfd-style pairwise interaction, forward and adjoint (the
                paper names the interaction's inputs in Section 3.1 but gives no
                formula; the formula here is this project's reading).
* ``spmv``    - y_i += w * x_j over the bipartite SpMV graph (Section 5.2).
* ``baselines`` - PowerGraph's random and greedy vertex-cut placements, the
                partitioners the paper compares against (Section 3.3).
* ``brute``   - exhaustive optimal partitions for tiny graphs (Theorems 1-2).
* ``hub``     - the hub split before the EP order (an extension for power-law
                graphs, not in the paper; pinned on ``hub_split7.json``, by its
                reduction to the plain EP order and by invariants).

Parity status: the cost, transform, flux, adjoint and SpMV functions are pinned
by closed forms, invariants, textbook properties and library routines in the
CPU tests; the tolerance floors (``flux.forward_abs``, ``flux.backward_abs``)
and the signed forward are pinned on one hand-derived edge.  ``cpack.layout``
is plain first-touch packing and pinned by that definition recomputed in the
tests and on a hand-derived three-part case (``cpack_three_parts.json``); the
library orders each owned range differently (by the next part touching a
vertex) and is compared with it through the owned ranges, owned and foreign
vertex sets and the isolated tail, which both orderings share.  The
partitioners are pinned exactly on hand-derived cases under tests/golden/:
``multilevel.partition`` and ``ggp.partition`` on Figure 1 (``fig1.json``, whose optimum is unique up to part labels), on a path
whose edge ids run out of path order (``multilevel_path9.json``) and on graphs
where refinement moves a node and where the contiguity pass moves a piece
(``multilevel_refine5.json``, ``multilevel_contiguity6.json``), with one
coarsening level pinned on small weighted graphs in the tests;
``baselines.greedy_partition`` on a 9-edge case (``greedy_vertex_cut9.json``).
Each step of these heuristics (seeding, growing, matching, refinement,
contiguity, greedy placement) is pinned by one of those cases.  On larger
graphs their exact output has no value independent of those steps; there the
library is compared with the oracle bit for bit.
"""

from . import graph, cost, ggp, multilevel, cpack, flux, spmv, brute, baselines, hub  # noqa: F401


def partition(edges, n, cap, order="ep", class_weight=None, n_x=0, hub_degree=0):
    """(part, task_order) for an order: 'ep' (multilevel, the default), 'ggp'
    (single-pass greedy growing), 'input' (consecutive blocks), or the
    baselines 'random' and 'greedy'.  class_weight (EP only): per-class vertex
    weights (x: ids below n_x, y: the rest).  hub_degree > 0 (EP only): the hub
    split first."""
    if order == "ep" and hub_degree > 0:
        part, task, _ = hub.partition(edges, n, cap, hub_degree, class_weight, n_x)
        return part, task
    if order == "ep":
        part, task, _ = multilevel.partition(edges, n, cap, class_weight, n_x)
        return part, task
    if order == "ggp":
        return ggp.partition(edges, n, cap, order="ep")
    if order == "random":
        return baselines.random_partition(len(edges), cap)
    if order == "greedy":
        return baselines.greedy_partition(edges, n, cap)
    return ggp.partition(edges, n, cap, order="input")

"""Adaptive overhead control on the host: background partition, reuse pre-check,
hand-over and cancellation (C ABI through the binding; no GPU needed)."""

import time

import numpy as np
import pytest

import gen
from oracle import cost

epk = pytest.importorskip("paper_1605_02043_amd")
from paper_1605_02043_amd.adaptive import AdaptivePartition  # noqa: E402
from paper_1605_02043_amd.plan import partition  # noqa: E402


def _bound(edges, n, cap):
    """1 - n_active / L_input from the oracle's cost of the default order."""
    m = len(edges)
    part = np.arange(m) // cap
    c = cost.partition_cost(edges, n, part, -(-m // cap))
    return 1.0 - c["n_active"] / c["loads"]


def test_ready_plan_equals_direct_partition():
    G = gen.grid2d(40, 30, seed=4)
    a = AdaptivePartition(G["edges"], G["n"], 64, G["geom"].astype(np.float32))
    P = a.take(wait=True)
    info = a.poll()
    assert info["state"] == "ready" and info["seconds"] > 0
    assert info["saving_bound"] == pytest.approx(_bound(G["edges"], G["n"], 64), rel=1e-12)
    part, task = P.part_of_edge()
    p2, t2, _ = partition(G["edges"], G["n"], 64, "ep")
    assert np.array_equal(part, p2) and np.array_equal(task, t2)
    with pytest.raises(epk.EpkError, match="already taken"):
        a.take(wait=True)
    a.close()


def test_precheck_skips_graph_without_reuse():
    # a perfect matching: every vertex has one edge, so no order can save a load
    n = 200
    E = np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], 1)
    geom = np.tile([1.0, 0.0, 0.0, 1.0], (len(E), 1)).astype(np.float32)
    a = AdaptivePartition(E, n, 16, geom, min_saving=0.05)
    assert a.poll()["state"] == "skipped" and a.poll()["saving_bound"] == 0.0
    assert a.take(wait=True) is None
    a.close()


def test_cancel_returns_promptly():
    T = gen.tet_mesh(40, 40, 40, seed=0)
    t0 = time.perf_counter()
    a = AdaptivePartition(T["edges"], T["n"], 256, T["geom"].astype(np.float32), min_saving=0.0)
    started = time.perf_counter() - t0
    assert a.poll()["state"] in ("running", "ready")
    t1 = time.perf_counter()
    a.close()  # cancels at the next coarsening level or refinement pass
    assert time.perf_counter() - t1 < 10.0 + started

"""Pins for the oracle's partition side: Definitions 1-4, Eq. 1, Theorems 1-2,
Figure 1 / Figure 3, closed forms and brute force on tiny graphs."""

import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import brute, cost, cpack, ggp, graph


def _fig1(golden_dir):
    with open(os.path.join(golden_dir, "fig1.json")) as f:
        return json.load(f)


def _fetched_twice(edges, n, part):
    return cost.partition_cost(edges, n, part)["replicated"]


# ---------------------------------------------------------------- Figure 1 / 3

def test_fig1_default_schedule_loads(golden_dir):
    G = _fig1(golden_dir)
    E, n, T = np.array(G["edges"]), G["n"], G["threads_per_block"]
    part = np.arange(len(E)) // T  # consecutive tasks per block
    assert part.tolist() == G["default_parts"]
    c = cost.partition_cost(E, n, part)
    assert c["loads"] == G["default_loads"] == 9
    assert cost.loads_simple(E, part) == 9
    assert _fetched_twice(E, n, part) == G["default_fetched_twice"] == 3


def test_fig1_ep_schedule_loads(golden_dir):
    G = _fig1(golden_dir)
    E, n = np.array(G["edges"]), G["n"]
    c = cost.partition_cost(E, n, G["ep_parts"])
    assert c["loads"] == G["ep_loads"] == 7
    assert c["cost"] == G["optimal_cost"] == 1
    assert _fetched_twice(E, n, G["ep_parts"]) == G["ep_fetched_twice"] == 1
    # the particle shared by e1, e2, e4 lands in one block only
    assert c["p_v"][G["ep_shared_by_e1_e2_e4_loaded_once"]] == 1


def test_fig1_brute_force_optimum(golden_dir):
    G = _fig1(golden_dir)
    E, n = np.array(G["edges"]), G["n"]
    best, _ = brute.min_edge_partition_cost(E, n, G["threads_per_block"])
    assert best == G["optimal_cost"]


def test_cpack_hand_derived_three_parts(golden_dir):
    """cpack.layout against a case derived by hand (tests/golden/cpack_three_parts.json):
    three parts sharing vertices in both directions, owned ranges in first-touch order,
    foreign lists ascending, an isolated vertex last."""
    with open(os.path.join(golden_dir, "cpack_three_parts.json")) as f:
        G = json.load(f)
    E = np.array(G["edges"])
    lay = cpack.layout(E, G["n"], G["part"], G["task"])
    assert lay["perm"].tolist() == G["perm"]
    for p, info in enumerate(lay["parts"]):
        assert info["own0"][0] == G["own_begin"][p] and info["nown"][0] == G["own_count"][p]
        assert list(info["foreign"][0]) == G["foreign"][p]
    c = cost.partition_cost(E, G["n"], np.array(G["part"]), 3)
    assert (c["loads"], c["cost"], c["replicated"], c["slots"]) == (G["loads"], G["cost"], G["replicated"], G["slots"])


def test_fig1_ggp_finds_the_ep_schedule(golden_dir):
    G = _fig1(golden_dir)
    E, n = np.array(G["edges"]), G["n"]
    part, task = ggp.partition(E, n, G["threads_per_block"])
    assert part.tolist() == G["ep_parts"]
    assert task.tolist() == [0, 1, 3, 2, 4, 5]
    assert cost.partition_cost(E, n, part)["loads"] == 7


# ---------------------------------------------------------------- Definition 3 counts

def _random_graph(rng, n, m, allow_dup=True):
    E = []
    while len(E) < m:
        u, v = rng.integers(0, n, 2)
        if u == v:
            continue
        if not allow_dup and (min(u, v), max(u, v)) in {(min(a, b), max(a, b)) for a, b in E}:
            continue
        E.append((int(u), int(v)))
    return np.array(E, dtype=np.int64).reshape(-1, 2)


@settings(max_examples=40, deadline=None)
@given(st.integers(2, 12), st.integers(1, 30), st.integers(0, 10_000))
def test_transform_counts(n, m, seed):
    E = _random_graph(np.random.default_rng(seed), n, m)
    D = graph.clone_and_connect(E, n)
    deg = np.bincount(E.ravel(), minlength=n)
    n_active = int((deg > 0).sum())
    assert D["n_clones"] == 2 * m  # |V'| = 2m
    assert len(D["aux"]) == int((deg[deg > 0] - 1).sum()) == 2 * m - n_active
    # every clone is on exactly one original edge
    on = np.zeros(2 * m, dtype=int)
    for a, b in D["original"]:
        on[a] += 1
        on[b] += 1
    assert (on == 1).all()
    # the clones of each vertex form a path: degree <= 2 in the aux graph, d-1 links
    adeg = np.zeros(2 * m, dtype=int)
    for a, b in D["aux"]:
        assert D["owner"][a] == D["owner"][b]
        adeg[a] += 1
        adeg[b] += 1
    assert adeg.max(initial=0) <= 2
    # contracted links are the aux edges seen from each contracted node
    nbr = graph.contracted_links(E, n)
    assert sum(len(x) for x in nbr) == 2 * len(D["aux"])


def test_reconstruct_rejects_cut_original_edge():
    E = np.array([[0, 1], [1, 2]])
    D = graph.clone_and_connect(E, 3)
    with pytest.raises(ValueError):
        graph.reconstruct(D, [0, 1, 0, 0])
    assert graph.reconstruct(D, [1, 1, 0, 0]).tolist() == [1, 0]


# ---------------------------------------------------------------- invariants of the partitioner

@settings(max_examples=60, deadline=None)
@given(st.integers(2, 40), st.integers(1, 120), st.integers(1, 17), st.integers(0, 10_000))
def test_ggp_invariants(n, m, cap, seed):
    E = _random_graph(np.random.default_rng(seed), n, m)
    part, task = ggp.partition(E, n, cap)
    k = math.ceil(m / cap)
    assert sorted(task.tolist()) == list(range(m))  # every edge placed exactly once
    sizes = np.bincount(part, minlength=k)
    assert len(sizes) == k and part.min() == 0 and part.max() == k - 1
    assert (sizes[:-1] == cap).all() and 1 <= sizes[-1] <= cap
    # task order visits the parts in ascending id
    assert (np.diff(part[task]) >= 0).all()
    c = cost.partition_cost(E, n, part, k)
    assert c["loads"] == c["cost"] + c["n_active"]
    assert c["slots"] == c["cost"] + c["replicated"]
    assert c["loads"] == cost.loads_simple(E, part)
    # Theorem 1: cut auxiliary edges bound the vertex-cut cost
    assert c["cost"] <= c["aux_cut"]
    D = graph.clone_and_connect(E, n)
    assert graph.vertex_cut(D, np.repeat(part, 2)) == c["aux_cut"]
    # the layout's per-part vertex lists add up to the loads
    lay = cpack.layout(E, n, part, task)
    assert sum(info["nown"][0] + len(info["foreign"][0]) for info in lay["parts"]) == c["loads"]
    assert sum(len(info["foreign"][0]) for info in lay["parts"]) == c["cost"]


@settings(max_examples=40, deadline=None)
@given(st.integers(2, 30), st.integers(1, 80), st.integers(1, 9), st.integers(0, 10_000))
def test_theorem2_rechained_transform_is_exact(n, m, cap, seed):
    """Regrouping each vertex's clones by part makes the aux cut equal C."""
    E = _random_graph(np.random.default_rng(seed), n, m)
    for part in (ggp.partition(E, n, cap)[0], np.arange(m) // cap,
                 np.random.default_rng(seed + 1).integers(0, math.ceil(m / cap), m)):
        D2 = graph.rechain_by_part(E, n, part)
        assert graph.vertex_cut(D2, np.repeat(part, 2)) == cost.partition_cost(E, n, part)["cost"]


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_bounds(seed):
    """C* <= C(GGP); C* <= C(recon(VP*)) <= cut(VP*) <= (d_max - 1) C*  (Theorems 1-2)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 7))
    m = int(rng.integers(3, 9))
    cap = int(rng.integers(2, 5))
    E = _random_graph(rng, n, m)
    c_star, _ = brute.min_edge_partition_cost(E, n, cap)
    cut_star, vp_part = brute.min_vertex_partition_cut(E, n, cap)
    c_recon = cost.partition_cost(E, n, vp_part)["cost"]
    d_max = int(np.bincount(E.ravel()).max())
    assert c_star <= c_recon <= cut_star <= max(d_max - 1, 1) * c_star or (c_star == 0 and cut_star == 0)
    part, _ = ggp.partition(E, n, cap)
    assert cost.partition_cost(E, n, part)["cost"] >= c_star


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("m,cap", [(1, 1), (10, 3), (64, 8), (65, 8), (200, 16)])
def test_path_closed_form(m, cap):
    E = np.stack([np.arange(m), np.arange(1, m + 1)], axis=1)
    k = math.ceil(m / cap)
    part, _ = ggp.partition(E, m + 1, cap)
    assert cost.partition_cost(E, m + 1, part)["cost"] == k - 1
    if m <= 9:
        assert brute.min_edge_partition_cost(E, m + 1, cap)[0] == k - 1


@pytest.mark.parametrize("m,cap", [(1, 1), (9, 4), (30, 7), (100, 10)])
def test_star_closed_form(m, cap):
    E = np.stack([np.zeros(m, dtype=int), np.arange(1, m + 1)], axis=1)
    k = math.ceil(m / cap)
    rng = np.random.default_rng(m)
    for part in (ggp.partition(E, m + 1, cap)[0], np.arange(m) // cap, rng.permutation(np.arange(m) // cap)):
        assert cost.partition_cost(E, m + 1, part)["cost"] == k - 1


@pytest.mark.parametrize("m,cap", [(6, 3), (8, 2), (9, 4)])
def test_cycle_closed_form(m, cap):
    E = np.stack([np.arange(m), (np.arange(m) + 1) % m], axis=1)
    k = math.ceil(m / cap)
    assert brute.min_edge_partition_cost(E, m, cap)[0] == k
    part, _ = ggp.partition(E, m, cap)
    assert cost.partition_cost(E, m, part)["cost"] >= k


@pytest.mark.parametrize("seed", range(5))
def test_disjoint_components_reach_zero(seed):
    cap = 6
    rng = np.random.default_rng(seed)
    comps = []
    base = 0
    for _ in range(7):  # components of exactly cap edges: paths, stars, a triangle fan
        kind = rng.integers(0, 3)
        if kind == 0:
            comps.append(np.stack([np.arange(cap), np.arange(1, cap + 1)], 1) + base)
            base += cap + 1
        elif kind == 1:
            comps.append(np.stack([np.zeros(cap, int), np.arange(1, cap + 1)], 1) + base)
            base += cap + 1
        else:
            comps.append(np.array([[0, 1], [1, 2], [0, 2], [2, 3], [0, 3], [3, 4]]) + base)
            base += 5
    E = np.concatenate(comps)
    ids = rng.permutation(base)
    E = ids[E]
    E = E[rng.permutation(len(E))]
    part, _ = ggp.partition(E, base, cap)
    assert cost.partition_cost(E, base, part)["cost"] == 0


@settings(max_examples=30, deadline=None)
@given(st.integers(1, 60), st.integers(1, 10), st.integers(0, 1000))
def test_max_degree_two_aux_cut_equals_cost(m, cap, seed):
    """Disjoint paths and cycles (d_max <= 2): every cut chain link is a split vertex."""
    rng = np.random.default_rng(seed)
    n = 2 * m + 2
    ids = rng.permutation(n)
    E = []
    v = 0
    while len(E) < m:
        L = int(rng.integers(1, 8))
        L = min(L, m - len(E))
        for t in range(L):
            E.append((ids[v + t], ids[v + t + 1]))
        v += L + 1
    E = np.array(E)
    E = E[rng.permutation(len(E))]
    for part in (ggp.partition(E, n, cap)[0], rng.integers(0, math.ceil(m / cap), m)):
        c = cost.partition_cost(E, n, part)
        assert c["aux_cut"] == c["cost"]


def test_input_order_is_consecutive_blocks():
    E = _random_graph(np.random.default_rng(3), 20, 50)
    part, task = ggp.partition(E, 20, 7, order="input")
    assert part.tolist() == (np.arange(50) // 7).tolist()
    assert task.tolist() == list(range(50))


# ---------------------------------------------------------------- cpack

@settings(max_examples=40, deadline=None)
@given(st.integers(2, 40), st.integers(1, 100), st.integers(1, 13), st.integers(0, 1000))
def test_cpack_layout(n, m, cap, seed):
    E = _random_graph(np.random.default_rng(seed), n, m)
    part, task = ggp.partition(E, n, cap)
    lay = cpack.layout(E, n, part, task)
    perm = lay["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    assert (lay["orig_to_packed"][perm] == np.arange(n)).all()
    # packed ids in the order of first touch along the task sequence (u then v of
    # each edge), isolated vertices last in ascending id
    seen, order = set(), []
    for e in task:
        for w in E[e]:
            if int(w) not in seen:
                seen.add(int(w))
                order.append(int(w))
    iso = sorted(set(range(n)) - seen)
    assert perm.tolist() == order + iso
    # owned ranges tile [0, n_active) in part order
    cur = 0
    for info in lay["parts"]:
        assert info["own0"][0] == cur
        cur += info["nown"][0]
        f = info["foreign"][0]
        assert (np.diff(f) > 0).all() if len(f) > 1 else True
        assert (f < info["own0"][0]).all()  # foreign vertices were packed by earlier parts
    assert cur == n - len(iso)


def test_cpack_bipartite_classes():
    rng = np.random.default_rng(7)
    n_x, n_y = 30, 20
    m = 90
    E = np.stack([rng.integers(0, n_x, m), n_x + rng.integers(0, n_y, m)], 1)
    part, task = ggp.partition(E, n_x + n_y, 8)
    lay = cpack.layout(E, n_x + n_y, part, task, n_x=n_x)
    o2p = lay["orig_to_packed"]
    assert (o2p[:n_x] < n_x).all() and (o2p[n_x:] >= n_x).all()
    c = cost.partition_cost(E, n_x + n_y, part)
    tot = sum(info["nown"][cl] + len(info["foreign"][cl]) for info in lay["parts"] for cl in (0, 1))
    assert tot == c["loads"]


# ---------------------------------------------------------------- multilevel (the EP order)

from oracle import multilevel  # noqa: E402


def test_multilevel_fig1(golden_dir):
    G = _fig1(golden_dir)
    E, n = np.array(G["edges"]), G["n"]
    part, task, k = multilevel.partition(E, n, G["threads_per_block"])
    assert k == 2
    assert cost.partition_cost(E, n, part, k)["loads"] == G["ep_loads"] == 7
    # every split into two parts of 3 edges, enumerated: the cost-1 optimum is unique up to
    # the part labels, so the output is fixed exactly once labelled (the part holding edge 0
    # is part 0; edge ids ascend inside a part)
    import itertools

    optima = []
    for first in itertools.combinations(range(6), 3):
        p = np.ones(6, dtype=np.int64)
        p[list(first)] = 0
        loads = sum(len({int(w) for e in range(6) if p[e] == q for w in E[e]}) for q in (0, 1))
        if loads == 7:
            optima.append(p.tolist())
    assert sorted(optima) == sorted([G["ep_parts"], [1 - x for x in G["ep_parts"]]])
    assert part.tolist() == G["ep_parts"]
    assert task.tolist() == [0, 1, 3, 2, 4, 5]


def test_multilevel_and_ggp_hand_derived_path(golden_dir):
    """A path whose edge ids are out of path order (tests/golden/multilevel_path9.json): the
    second part must start from the node most linked to placed nodes, not from the smallest
    unplaced id, which would swap the last two part labels.  Derived by hand from the growing
    rules; both partitioners grow the same parts."""
    import json

    G = json.load(open(os.path.join(golden_dir, "multilevel_path9.json")))
    E, n, cap = np.array(G["edges"]), G["n"], G["capacity"]
    part, task, k = multilevel.partition(E, n, cap)
    assert k == G["k"] and part.tolist() == G["ep_parts"] and task.tolist() == G["ep_task_order"]
    c = cost.partition_cost(E, n, part, k)
    assert c["loads"] == G["loads"] and c["cost"] == G["cost"]
    gp, gt = ggp.partition(E, n, cap)
    assert gp.tolist() == G["ggp_parts"] and gt.tolist() == G["ggp_task_order"]


def test_multilevel_refinement_hand_derived(golden_dir):
    """A 5-edge graph where refinement moves one node and lowers the cost from 4 to 3
    (tests/golden/multilevel_refine5.json, derived by hand): the grown parts, the refined
    result of the multilevel order and the unrefined result of single-pass growing."""
    import json

    G = json.load(open(os.path.join(golden_dir, "multilevel_refine5.json")))
    E, n, cap = np.array(G["edges"]), G["n"], G["capacity"]
    k, target, _ = multilevel.parameters(len(E), cap)
    adj, w = multilevel._finest(E, n)
    grown = multilevel.grow(adj, w, k, target, cap)
    assert k == G["k"] and grown == G["grown_parts"]
    assert cost.partition_cost(E, n, np.array(grown), k)["loads"] == G["grown_loads"]
    part, task, k = multilevel.partition(E, n, cap)
    assert part.tolist() == G["ep_parts"] and task.tolist() == G["ep_task_order"]
    c = cost.partition_cost(E, n, part, k)
    assert c["loads"] == G["loads"] and c["cost"] == G["cost"]
    gp, gt = ggp.partition(E, n, cap)
    assert gp.tolist() == G["ggp_parts"] and gt.tolist() == G["ggp_task_order"]


def test_multilevel_contiguity_hand_derived(golden_dir):
    """A 6-edge multigraph where refinement splits a part in two pieces and the contiguity pass
    moves the lighter-id piece away, lowering the cost from 2 to 1
    (tests/golden/multilevel_contiguity6.json, derived by hand), step by step."""
    import json

    G = json.load(open(os.path.join(golden_dir, "multilevel_contiguity6.json")))
    E, n, cap = np.array(G["edges"]), G["n"], G["capacity"]
    k, target, _ = multilevel.parameters(len(E), cap)
    adj, w = multilevel._finest(E, n)
    p = multilevel.grow(adj, w, k, target, cap)
    assert p == G["grown_parts"]
    p = multilevel.refine(adj, w, p, k, cap)
    assert p == G["refined_parts"]
    p = multilevel.contiguity(adj, w, p, k, cap)
    assert p == G["ep_parts"]
    part, task, k = multilevel.partition(E, n, cap)
    assert part.tolist() == G["ep_parts"] and task.tolist() == G["ep_task_order"]
    c = cost.partition_cost(E, n, part, k)
    assert c["loads"] == G["loads"] and c["cost"] == G["cost"]
    gp, gt = ggp.partition(E, n, cap)
    assert gp.tolist() == G["ggp_parts"] and gt.tolist() == G["ggp_task_order"]


def test_coarsen_matching_rules_hand_derived():
    """One level of heavy-edge matching on small weighted graphs, derived by hand: nodes in
    ascending id take the unmatched neighbour of largest link weight (not the smallest id),
    within the coarse-node weight cap, ties to the smaller id; coarse ids follow the visit;
    node weights and link weights add and links inside a coarse node vanish."""
    adj = [{1: 1, 2: 3}, {0: 1, 3: 2}, {0: 3, 4: 1}, {1: 2}, {2: 1}]
    # 0 takes 2 (link 3 beats link 1), 1 takes 3, 4 has no unmatched neighbour left
    cadj, cw, cmap = multilevel.coarsen(adj, [1] * 5, 2)
    assert cmap == [0, 1, 0, 1, 2] and cw == [2, 2, 1]
    assert cadj == [{1: 1, 2: 1}, {0: 1}, {0: 1}]
    # node 2 weighs 2: 0 + 2 would exceed the cap, so 0 takes 1; 2, 3 and 4 stay single
    cadj, cw, cmap = multilevel.coarsen(adj, [1, 1, 2, 1, 1], 2)
    assert cmap == [0, 0, 1, 2, 3] and cw == [2, 2, 1, 1]
    assert cadj == [{1: 3, 2: 2}, {0: 3, 3: 1}, {0: 2}, {1: 1}]
    # equal link weights: the smaller id wins
    cadj, cw, cmap = multilevel.coarsen([{3: 1, 1: 1}, {0: 1}, {}, {0: 1}], [1] * 4, 2)
    assert cmap == [0, 0, 1, 2] and cw == [2, 1, 1] and cadj == [{2: 1}, {}, {0: 1}]


@settings(max_examples=60, deadline=None)
@given(st.integers(2, 40), st.integers(1, 150), st.integers(1, 40), st.integers(0, 10_000))
def test_multilevel_invariants(n, m, cap, seed):
    E = _random_graph(np.random.default_rng(seed), n, m)
    part, task, k = multilevel.partition(E, n, cap)
    assert k == math.ceil(m / (cap - cap // 20))
    assert sorted(task.tolist()) == list(range(m))
    assert part.min() >= 0 and part.max() < k
    sizes = np.bincount(part, minlength=k)
    assert sizes.max() <= cap  # hard capacity
    pt = part[task]
    assert (np.diff(pt) >= 0).all()  # parts in ascending order
    for p in range(k):  # ascending edge id inside a part
        ids = task[pt == p]
        assert (np.diff(ids) > 0).all()
    c = cost.partition_cost(E, n, part, k)
    assert c["balance"] <= cap / (m / k) + 1e-12
    assert c["cost"] <= c["aux_cut"]  # Theorem 1
    assert c["loads"] == c["cost"] + c["n_active"]


def test_multilevel_capacity_regression_no_room():
    """Below cap 20 the capacity leaves no room above the growth target (k = ceil(m/cap)).
    Coarse nodes of weight 2 then stalled growth one short of the target and the rest
    overflowed a part (this graph gave a part of 18 edges at cap 17).  The node-weight
    bound (room + 1, so 1 here) keeps every part within the capacity (Eq. 1, Section 3.2)."""
    E = _random_graph(np.random.default_rng(0), 2, 146)
    assert multilevel.max_node_weight(17) == 1
    part, task, k = multilevel.partition(E, 2, 17)
    assert k == 9 and np.bincount(part, minlength=k).max() <= 17
    assert sorted(task.tolist()) == list(range(146))


@pytest.mark.parametrize("cap", [1, 5, 16, 17, 18, 19, 20, 21, 39, 40, 63, 64, 127, 256, 512, 1024])
def test_multilevel_node_weight_within_room(cap):
    """The coarse-node weight bound never exceeds the room above the target plus one,
    so a part below the target always fits the next node; from cap 20 up it is the
    plain max(2, cap/32) rule."""
    w = multilevel.max_node_weight(cap)
    assert 1 <= w <= cap // 20 + 1
    if cap >= 20:
        assert w == max(2, cap // 32)


@pytest.mark.parametrize("seed", range(10))
def test_multilevel_not_below_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 7))
    m = int(rng.integers(3, 9))
    cap = int(rng.integers(2, 5))
    E = _random_graph(rng, n, m)
    part, _, k = multilevel.partition(E, n, cap)
    assert k == math.ceil(m / cap)  # cap < 20: no room below the capacity
    c_star, _ = brute.min_edge_partition_cost(E, n, cap)
    assert cost.partition_cost(E, n, part, k)["cost"] >= c_star


@pytest.mark.parametrize("m,cap", [(10, 3), (64, 8), (200, 16), (1000, 40)])
def test_multilevel_path_is_optimal(m, cap):
    """A path split into q nonempty parts costs at least q - 1; contiguous arcs reach it."""
    E = np.stack([np.arange(m), np.arange(1, m + 1)], axis=1)
    part, _, k = multilevel.partition(E, m + 1, cap)
    q = len(np.unique(part))
    assert cost.partition_cost(E, m + 1, part, k)["cost"] == q - 1


def test_multilevel_components_reach_zero():
    cap = 6
    rng = np.random.default_rng(4)
    comps, base = [], 0
    for _ in range(9):
        comps.append(np.stack([np.arange(cap), np.arange(1, cap + 1)], 1) + base)
        base += cap + 1
    E = np.concatenate(comps)
    E = rng.permutation(base)[E]
    E = E[rng.permutation(len(E))]
    part, _, k = multilevel.partition(E, base, cap)
    assert cost.partition_cost(E, base, part, k)["cost"] == 0


def test_multilevel_beats_single_pass_on_meshes():
    """Not a pin of exact output: the multilevel order must not load more than greedy growing."""
    import gen

    for G in (gen.grid2d(40, 30, seed=2), gen.tet_mesh(10, 9, 8, seed=2)):
        E, n = G["edges"], G["n"]
        pm, _, k = multilevel.partition(E, n, 128)
        pg, _ = ggp.partition(E, n, 128)
        assert cost.partition_cost(E, n, pm, k)["loads"] < cost.partition_cost(E, n, pg)["loads"]


# ------------------------------------------------------------------ baselines (PowerGraph vertex cuts)

def test_splitmix64_published_values():
    """The first outputs of SplitMix64 seeded with 0 (the generator's published sequence)."""
    from oracle.baselines import splitmix64

    g = 0x9E3779B97F4A7C15
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    assert splitmix64(g) == 0x6E789E6AA1B965F4
    assert splitmix64(2 * g % (1 << 64)) == 0x06C45D188009454F


@pytest.mark.parametrize("m,cap", [(0, 4), (1, 4), (17, 4), (64, 8), (100, 7)])
def test_random_baseline_is_balanced_permutation(m, cap):
    from oracle.baselines import random_partition

    part, task = random_partition(m, cap)
    assert sorted(task.tolist()) == list(range(m))
    k = -(-m // cap)
    sizes = np.bincount(part, minlength=k) if m else np.zeros(0, int)
    assert all(sizes[:-1] == cap) if k > 1 else True
    assert (part[task] == np.arange(m) // cap).all()


@pytest.mark.parametrize("name", ["greedy_vertex_cut9.json", "greedy_tie5.json"])
def test_greedy_baseline_hand_derived(golden_dir, name):
    """Greedy vertex-cut placement on small graphs derived by hand: a 9-edge graph
    (greedy_vertex_cut9.json: shared part, the endpoint with more unplaced edges, one placed
    endpoint, and the fall-back to the least loaded part when the preferred parts are full),
    and a 5-edge graph whose endpoints tie on unplaced edges (greedy_tie5.json: the first
    endpoint's parts win)."""
    import json

    from oracle.baselines import greedy_partition

    G = json.load(open(os.path.join(golden_dir, name)))
    E = np.array(G["edges"])
    part, task = greedy_partition(E, G["n"], G["capacity"])
    assert part.tolist() == G["greedy_parts"] and task.tolist() == G["greedy_task_order"]
    c = cost.partition_cost(E, G["n"], part, G["k"])
    assert c["loads"] == G["loads"] and c["cost"] == G["cost"]


def test_greedy_baseline_capacity_and_closed_forms():
    from oracle.baselines import greedy_partition

    # disjoint components of exactly cap edges, listed one after another: cost 0
    cap, comps = 6, 5
    E = []
    for c in range(comps):
        base = 10 * c
        E += [(base + i, base + i + 1) for i in range(cap)]  # a path of cap edges
    E = np.array(E)
    part, task = greedy_partition(E, 10 * comps, cap)
    assert cost.partition_cost(E, 10 * comps, part, comps)["cost"] == 0
    # a path in order: consecutive blocks, the optimum k - 1
    P = np.array([(i, i + 1) for i in range(40)])
    part, _ = greedy_partition(P, 41, 8)
    assert cost.partition_cost(P, 41, part, 5)["cost"] == 4
    # a star: every part holds the hub, cost k - 1 whatever the placement
    S = np.array([(0, i) for i in range(1, 30)])
    part, _ = greedy_partition(S, 30, 4)
    assert np.bincount(part).max() <= 4
    assert cost.partition_cost(S, 30, part, 8)["cost"] == 7


def test_baselines_rank_below_ep_on_a_mesh():
    """Sanity, not a pin: on a 2D mesh the transform-based order beats greedy, which beats random."""
    import gen
    import oracle

    G = gen.grid2d(24, 24, seed=0)
    k = {}
    for order in ("ep", "greedy", "random"):
        part, _ = oracle.partition(G["edges"], G["n"], 64, order)
        k[order] = cost.partition_cost(G["edges"], G["n"], part, int(part.max()) + 1)["cost"]
    assert k["ep"] < k["greedy"] < k["random"]


# ---------------------------------------------------------------- per-class vertex weights

# A hand-derived case: x vertices 0, 1 and y vertices 2, 3 (n_x = 2), edges
# e0 = (x0, y0), e1 = (x0, y1), e2 = (x1, y0), e3 = (x1, y1), capacity 2 (k = 2, no coarsening).
# Chains: x0 links e0-e1, x1 links e2-e3, y0 links e0-e2, y1 links e1-e3.
# Uniform weights: growth starts at e0, whose links to e1 (x0) and e2 (y0) tie at 1, so the
#   smaller id e1 joins: parts {e0, e1} | {e2, e3}; both y vertices are replicated (C = 2).
# Weights (x 1, y 4): e2's link weighs 4, so e2 joins: parts {e0, e2} | {e1, e3}; both x vertices
#   are replicated, weighted cost 1 + 1 = 2 (the uniform split would cost 4 + 4 = 8).
_K22 = np.array([[0, 2], [0, 3], [1, 2], [1, 3]])


def test_weighted_multilevel_hand_derived():
    part, task, k = multilevel.partition(_K22, 4, 2)
    assert part.tolist() == [0, 0, 1, 1] and task.tolist() == [0, 1, 2, 3]
    part_w, task_w, _ = multilevel.partition(_K22, 4, 2, class_weight=(1, 4), n_x=2)
    assert part_w.tolist() == [0, 1, 0, 1] and task_w.tolist() == [0, 2, 1, 3]
    w = np.array([1, 1, 4, 4])
    assert cost.weighted_cost(_K22, 4, part, w) == 8 and cost.weighted_cost(_K22, 4, part_w, w) == 2
    best, _ = brute.min_edge_partition_cost(_K22, 4, 2, w)
    assert best == 2
    # uniform weights (1, 1) are the paper's cost: the same partition as no weights
    p1, t1, _ = multilevel.partition(_K22, 4, 2, class_weight=(1, 1), n_x=2)
    assert p1.tolist() == part.tolist() and t1.tolist() == task.tolist()


def test_weighted_cost_definitions():
    """weighted_cost with unit weights is C; weighted_aux_cut with unit weights is the aux cut."""
    rng = np.random.default_rng(5)
    E = _random_graph(rng, 12, 40)
    part = rng.integers(0, 5, 40)
    c = cost.partition_cost(E, 12, part)
    assert cost.weighted_cost(E, 12, part, np.ones(12)) == c["cost"]
    assert cost.weighted_aux_cut(E, part, np.ones(12)) == c["aux_cut"]


@settings(max_examples=40, deadline=None)
@given(st.integers(2, 15), st.integers(2, 15), st.integers(1, 120), st.integers(1, 30), st.integers(1, 8),
       st.integers(0, 10_000))
def test_weighted_multilevel_invariants_and_theorem1(n_x, n_y, m, cap, wy, seed):
    """Weighted EP on random bipartite graphs: every edge once within the capacity, and the
    weighted form of Theorem 1: sum_v w(v) (p_v - 1) <= the weighted cut of the transform."""
    rng = np.random.default_rng(seed)
    E = np.stack([rng.integers(0, n_x, m), n_x + rng.integers(0, n_y, m)], 1)
    part, task, k = multilevel.partition(E, n_x + n_y, cap, class_weight=(1, wy), n_x=n_x)
    assert sorted(task.tolist()) == list(range(m))
    assert np.bincount(part, minlength=k).max() <= cap
    w = np.array([1] * n_x + [wy] * n_y)
    assert cost.weighted_cost(E, n_x + n_y, part, w) <= cost.weighted_aux_cut(E, part, w)


@pytest.mark.parametrize("seed", range(6))
def test_weighted_multilevel_not_below_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    n_x, n_y = int(rng.integers(2, 4)), int(rng.integers(2, 4))
    m = int(rng.integers(3, 8))
    cap = int(rng.integers(2, 4))
    E = np.stack([rng.integers(0, n_x, m), n_x + rng.integers(0, n_y, m)], 1)
    w = np.array([1] * n_x + [5] * n_y)
    part, _, k = multilevel.partition(E, n_x + n_y, cap, class_weight=(1, 5), n_x=n_x)
    best, _ = brute.min_edge_partition_cost(E, n_x + n_y, cap, w)
    assert cost.weighted_cost(E, n_x + n_y, part, w) >= best


# ------------------------------------------------------------------ the hub split (an extension)

from oracle import hub  # noqa: E402


def test_hub_split_hand_derived(golden_dir):
    """Both hand-derived cases: the bipartite one pins the sort by the other endpoint and the
    run of cap; the one-class one pins the key rule (larger degree, ties to the smaller id, an
    edge listed high id first) and the EP part of the rest following the hub parts."""
    G = json.load(open(os.path.join(golden_dir, "hub_split7.json")))
    for c in G["cases"]:
        part, task, k = hub.partition(c["edges"], c["n"], c["cap"], c["hub_degree"], None, c["n_x"])
        assert part.tolist() == c["part"], c["name"]
        assert task.tolist() == c["task"], c["name"]
        assert k == c["n_parts"], c["name"]


def _bipartite_power_law(rng, n_x, n_y, m, alpha=1.2):
    """Edges (x, n_x + y) with y drawn from a Zipf-like law, so that a few y have high degree."""
    py = 1.0 / np.arange(1, n_y + 1) ** alpha
    y = rng.choice(n_y, size=m, p=py / py.sum())
    x = rng.integers(0, n_x, m)
    return np.stack([x, n_x + y], 1).astype(np.int64)


@settings(max_examples=25, deadline=None)
@given(st.integers(2, 40), st.integers(2, 40), st.integers(1, 400), st.integers(1, 40), st.integers(1, 30),
       st.integers(0, 10_000))
def test_hub_split_invariants(n_x, n_y, m, cap, hd, seed):
    """Every edge in exactly one part, parts within the capacity and listed in ascending order by
    the task order; the hub parts hold exactly the hub edges, in (key, other, id) order; a hub
    of degree d spans at most ceil(d/cap) + 1 parts."""
    rng = np.random.default_rng(seed)
    E = _bipartite_power_law(rng, n_x, n_y, m)
    n = n_x + n_y
    part, task, k = hub.partition(E, n, cap, hd, None, n_x)
    assert sorted(task.tolist()) == list(range(m))
    assert (np.diff(part[task]) >= 0).all()
    counts = np.bincount(part, minlength=k)
    assert len(counts) == k and counts.max() <= cap
    deg = np.bincount(E.ravel(), minlength=n)
    is_hub = deg[E[:, 1]] > hd
    nh = int(is_hub.sum())
    kh = -(-nh // cap)
    assert (part[is_hub] < kh).all() and (part[~is_hub] >= kh).all()
    order = sorted(np.flatnonzero(is_hub).tolist(), key=lambda e: (E[e, 1], E[e, 0], e))
    assert task[:nh].tolist() == order
    for v in np.unique(E[is_hub, 1]):
        spans = len(np.unique(part[E[:, 1] == v]))
        assert spans <= -(-deg[v] // cap) + 1


@settings(max_examples=20, deadline=None)
@given(st.integers(2, 30), st.integers(0, 200), st.integers(1, 30), st.integers(0, 10_000))
def test_hub_split_without_hubs_is_the_ep_order(n, m, cap, seed):
    """With hub_degree at or above every degree the split finds no hub edge and the result is the
    plain EP order (weighted and unweighted, one class and two)."""
    rng = np.random.default_rng(seed)
    E = rng.integers(0, n, size=(m, 2))
    E = E[E[:, 0] != E[:, 1]]
    deg_max = int(np.bincount(E.ravel(), minlength=n).max()) if len(E) else 0
    for n_x, cw in ((0, None), (n // 2, (1, 3))):
        p1, t1, k1 = hub.partition(E, n, cap, max(deg_max, 1), cw, n_x)
        p2, t2, k2 = multilevel.partition(E, n, cap, cw, n_x)
        assert np.array_equal(p1, p2) and np.array_equal(t1, t2) and k1 == k2

"""C-ABI checks that need no GPU: every declared symbol is exported, host-only
entry points validate their inputs, and the C++ partitioner and packing agree
bit for bit with the oracle."""

import ctypes as C
import json
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import gen
from gen.rmat import spmv_graph
import oracle
from oracle import cost, cpack, ggp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

epk = pytest.importorskip("paper_1605_02043_amd")
from paper_1605_02043_amd import _lib  # noqa: E402
from paper_1605_02043_amd.plan import Plan, make_graph, partition  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "epk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epk_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 25
    raw = C.CDLL(_lib.LIB_PATH)
    for nm in names:
        assert hasattr(raw, nm), nm
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


def test_version_and_error_string():
    assert b"epk" in _lib.lib.epk_version()


def _status(fn, *args):
    return fn(*args)


def test_validation_errors():
    lib = _lib.lib
    part = np.zeros(4, dtype=np.int32)
    st = _lib.Stats()
    for edges, n, cap, code in [
        (np.array([[0, 1], [1, 1]]), 3, 2, _lib.EPK_EINVAL),  # self-loop
        (np.array([[0, 1], [1, 5]]), 3, 2, _lib.EPK_EINVAL),  # id out of range
        (np.array([[0, -1]]), 3, 2, _lib.EPK_EINVAL),
        (np.array([[0, 1]]), 3, 0, _lib.EPK_EINVAL),  # capacity < 1
    ]:
        gs, keep = make_graph(edges, n)
        s = lib.epk_partition(C.byref(gs), cap, 0, _lib.i32p(part), None, C.byref(st))
        assert s == code
        assert len(lib.epk_last_error()) > 0
    assert lib.epk_partition(None, 4, 0, _lib.i32p(part), None, C.byref(st)) == _lib.EPK_EINVAL
    gs, keep = make_graph(np.array([[0, 1]]), 2)
    assert lib.epk_partition(C.byref(gs), 4, 7, _lib.i32p(part), None, C.byref(st)) == _lib.EPK_EINVAL


def test_plan_errors():
    with pytest.raises(_lib.EpkError) as e:
        Plan(np.array([[0, 1]]), 2, 4, np.zeros((1, 3), np.float32))  # bad geometry width
    assert e.value.status == _lib.EPK_EINVAL
    with pytest.raises(_lib.EpkError) as e:
        Plan(np.array([[0, 1]]), 2, 4, np.ones(1, np.float32), kind="spmv", n_x=0)  # x/y classes wrong
    assert e.value.status == _lib.EPK_EINVAL
    with pytest.raises(_lib.EpkError) as e:
        Plan(np.array([[0, 1]]), 2, 4096, np.zeros((1, 4), np.float32))  # LDS budget
    assert e.value.status == _lib.EPK_ERANGE
    with pytest.raises(_lib.EpkError) as e:
        Plan(np.array([[0, 1]]), 2, 2048, np.ones(1, np.float32), kind="spmv", n_x=1)
    assert e.value.status == _lib.EPK_ERANGE


def test_lds_budget_boundary_on_tet32():
    """tet32 at capacity 896 fits the 64 KiB of LDS a workgroup may ask for (the adjoint's
    staging takes 99% of it, the GPU case of the largest capacity); at 1024 the plan is
    refused with EPK_ERANGE before anything touches a device."""
    import gen

    G = gen.workload("tet32", seed=0)
    P = Plan(G["edges"], G["n"], 896, G["geom"].astype(np.float32))
    assert 0.99 * 65536 <= P.info()["lds_bwd"] <= 65536
    with pytest.raises(_lib.EpkError) as e:
        Plan(G["edges"], G["n"], 1024, G["geom"].astype(np.float32))
    assert e.value.status == _lib.EPK_ERANGE and "LDS" in str(e.value)


@pytest.mark.parametrize("name,order,layout", [("tet", "ep", 0), ("tet", "ep", 1), ("tet", "input", 0),
                                               ("grid", "ep", 1), ("grid", "input", 0)])
def test_algorithmic_bytes_recounted(name, order, layout):
    """The roofline's numerators (epk_plan_info's algorithmic bytes), recounted here from the
    partition alone (loads, cost, replication from the oracle's cost function) with the bytes
    each kernel must move: the part kernels' edge records (4 + 4g per edge, g = 3 for the 3D
    area vector, 2 for the 2D normal), incidence lists (4 per edge), offsets (2 per local
    vertex and one more, each part's list padded to an even count), foreign ids (4 C), state
    gathers (20 L, 40 L for the adjoint's two row sets), owned rows (20 n_active) and partials
    (20 C), plus 32 bytes of header per part; the reduction's ids, offsets or records, partials
    and owner rows, and the zeroed untouched vertices."""
    import gen
    from oracle import cost

    G = gen.tet_mesh(6, 5, 4, seed=3) if name == "tet" else gen.workload("grid64", seed=1)
    E = np.asarray(G["edges"])
    n, m = G["n"], len(E)
    P = Plan(E, n, 64, G["geom"].astype(np.float32), order=order)
    P.set_slot_layout(layout)
    info, st, lay = P.info(), P.stats, P.layout()
    part, _ = P.part_of_edge()
    k = st["n_parts"]
    c = cost.partition_cost(E, n, part, k)
    L, C, R, na = c["loads"], c["cost"], c["replicated"], c["n_active"]
    assert (L, C, R) == (st["loads"], st["cost"], st["replicated"])
    U = lay["own_count"][:, 0].astype(np.int64) + np.diff(lay["foreign_offset"])
    assert U.sum() == L
    nloff = int(np.sum((U + 2) & ~1))
    g = 3 if G["geom"].shape[1] == 4 else 2
    meta = 32 * k + 4 * m + 4 * g * m + 4 * m + 2 * nloff + 4 * C
    ids = 4 * C if layout == 1 else 0
    fwd_kernel = meta + 20 * L + 20 * na + 20 * C + ids
    bwd_kernel = meta + 40 * L + 20 * na + 20 * C + ids
    red = 4 * R + 4 * (R + 1) + 20 * C + 40 * R + 20 * (n - na)
    if layout == 0:  # a 16-byte record per replicated vertex replaces its id and offsets
        ns = c["p_v"][c["p_v"] >= 2] - 1
        red += 16 * R - 4 * R - 4 * (R + 1) + int(np.sum(8 + 4 * ns[ns > 3]))
    assert info["vertex_major"] == layout
    assert (info["bytes_fwd_kernel"], info["bytes_bwd_kernel"]) == (fwd_kernel, bwd_kernel)
    assert (info["bytes_fwd"], info["bytes_bwd"]) == (fwd_kernel + red, bwd_kernel + red)


@pytest.mark.parametrize("layout", [0, 1])
def test_spmv_algorithmic_bytes_recounted(layout):
    """The same for SpMV: the part kernel reads 8 bytes per nonzero, 4 per foreign x id and per
    x load, writes 4 per active y (its owner's partial or its value) and per y partial; the
    reduction reads ids and offsets (or records), partials and owner values and writes the
    results, and zeroes the untouched y."""
    import gen
    from gen.rmat import spmv_graph
    from oracle import cost

    R_ = gen.rmat(scale=10, n_edges=1 << 13, seed=4)
    g = spmv_graph(R_, R_["shuffle"])
    E, n, n_x, m = np.asarray(g["edges"]), g["n"], g["n_x"], len(g["edges"])
    P = Plan(E, n, 64, g["w"], kind="spmv", n_x=n_x, class_weight=(1, 4), hub_degree=8)
    P.set_slot_layout(layout)
    info, st, lay = P.info(), P.stats, P.layout()
    part, _ = P.part_of_edge()
    k = st["n_parts"]
    pv = cost.partition_cost(E, n, part, k)["p_v"]
    fo = np.diff(lay["foreign_offset"]).reshape(k, 2)
    Cx, Cy = int(fo[:, 0].sum()), int(fo[:, 1].sum())
    Lx = int(lay["own_count"][:, 0].sum()) + Cx
    py = pv[n_x:]
    R, na = int(np.sum(py >= 2)), int(np.sum(py >= 1))
    assert Cy == int(np.sum(py[py >= 2] - 1))
    kernel = 32 * k + 8 * m + 4 * Cx + 4 * Lx + 4 * na + 4 * Cy + (4 * Cy if layout == 1 else 0)
    red = 4 * R + 4 * (R + 1) + 4 * Cy + 8 * R + 4 * (n - n_x - na)
    if layout == 0:
        ns = py[py >= 2] - 1
        red += 16 * R - 4 * R - 4 * (R + 1) + int(np.sum(8 + 4 * ns[ns > 3]))
    assert info["vertex_major"] == layout
    assert info["bytes_fwd_kernel"] == kernel and info["bytes_fwd"] == kernel + red


@pytest.mark.parametrize("cap,wg", [(1, 64), (64, 64), (128, 64), (256, 64), (300, 128), (1024, 256)])
def test_spmv_default_launch_four_edges_per_lane(cap, wg):
    """SpMV plans launch ceil(capacity / 4) lanes by default, rounded up to whole wavefronts:
    four edges per lane, the fastest shape on rmat20 once the kernel's loads are vectorised."""
    E = np.array([[j % 7, 7 + (j * 3) % 11] for j in range(40)], dtype=np.int32)
    P = Plan(E, 18, cap, np.ones(len(E), np.float32), kind="spmv", n_x=7)
    assert P.info()["wg"] == wg


def test_device_calls_refuse_before_upload():
    P = Plan(np.array([[0, 1], [1, 2]]), 3, 4, np.zeros((2, 4), np.float32))
    lib = _lib.lib
    assert lib.epk_forward(P._h, None, None, 0.0, None, None, None) == _lib.EPK_ESTATE
    assert lib.epk_backward(P._h, None, None, None, None, None) == _lib.EPK_ESTATE
    assert lib.epk_spmv(P._h, None, None, None, None) == _lib.EPK_ESTATE  # wrong kind
    ms = C.c_float(-1.0)
    assert lib.epk_run_stage_timed(P._h, 0, 0, None, None, None, 0.0, None, None, None, C.byref(ms)) == _lib.EPK_ESTATE
    assert ms.value == 0.0
    assert lib.epk_run_stage_timed(P._h, 0, 0, None, None, None, 0.0, None, None, None, None) == _lib.EPK_EINVAL
    assert lib.epk_run_stage_timed(P._h, 0, 2, None, None, None, 0.0, None, None, None, C.byref(ms)) == _lib.EPK_EINVAL
    with pytest.raises(_lib.EpkError):
        P.set_launch(wg=100)


# ------------------------------------------------------------------ parity with the oracle

def _check_parity(edges, n, cap, order="ep", n_x=None):
    part, task, st_ = partition(edges, n, cap, order)
    p2, t2 = oracle.partition(edges, n, cap, order)
    assert np.array_equal(part, p2) and np.array_equal(task, t2)
    c = cost.partition_cost(edges, n, p2, st_["n_parts"])
    for key in ("n_parts", "loads", "cost", "replicated", "slots", "aux_cut", "n_active", "max_part_edges",
                "max_part_vertices"):
        assert st_[key] == c[key], key
    assert st_["balance"] == pytest.approx(c["balance"], rel=1e-12)
    return part, task, p2, t2


@settings(max_examples=60, deadline=None)
@given(st.integers(2, 60), st.integers(0, 200), st.integers(1, 40), st.integers(0, 10_000),
       st.sampled_from(["ep", "ggp", "input", "random", "greedy"]))
def test_partition_parity_random(n, m, cap, seed, order):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    E = np.stack([u, v], 1).astype(np.int32)
    _check_parity(E, n, cap, order)


def test_partition_capacity_sweep_bit_equal():
    """Capacities 1-64 on small random multigraphs: the multilevel partition of the library
    equals the oracle's bit for bit and no part holds more than the capacity (Eq. 1 read as
    a hard capacity).  Sizes reach the coarsening regime (m > 16k) for every capacity from
    17 up, where weight-2 coarse nodes once overflowed parts at capacities 17-19."""
    rng = np.random.default_rng(20240)
    for cap in range(1, 65):
        for n, lo, hi in ((2, 16, 24), (7, 16, 24), (40, 16, 24), (40, 1, 16)):
            m = int(rng.integers(lo * cap, hi * cap))  # 16k < m from lo = 16 on
            u = rng.integers(0, n, m)
            v = (u + 1 + rng.integers(0, n - 1, m)) % n
            E = np.stack([u, v], 1).astype(np.int32)
            part, _, _, _ = _check_parity(E, n, cap, "ep")
            assert np.bincount(part).max() <= cap, (cap, n, m)


def test_partition_parity_grid64_and_fig1(golden_dir):
    G = gen.grid2d(64, 64, seed=0)
    for order in ("ep", "ggp", "input", "random", "greedy"):
        _check_parity(G["edges"], G["n"], 256, order)
    import json

    F = json.load(open(os.path.join(golden_dir, "fig1.json")))
    part, _, st_ = partition(np.array(F["edges"]), F["n"], 3)
    assert part.tolist() == F["ep_parts"] and st_["loads"] == 7
    part, _, st_ = partition(np.array(F["edges"]), F["n"], 3, "input")
    assert st_["loads"] == 9
    # the hand-derived path case: exact parts and task orders of both growing partitioners
    H = json.load(open(os.path.join(golden_dir, "multilevel_path9.json")))
    E = np.array(H["edges"])
    part, task, st_ = partition(E, H["n"], H["capacity"])
    assert part.tolist() == H["ep_parts"] and task.tolist() == H["ep_task_order"]
    assert st_["loads"] == H["loads"] and st_["cost"] == H["cost"] and st_["n_parts"] == H["k"]
    part, task, _ = partition(E, H["n"], H["capacity"], "ggp")
    assert part.tolist() == H["ggp_parts"] and task.tolist() == H["ggp_task_order"]
    for name in ("greedy_vertex_cut9.json", "greedy_tie5.json"):
        H = json.load(open(os.path.join(golden_dir, name)))
        part, task, st_ = partition(np.array(H["edges"]), H["n"], H["capacity"], "greedy")
        assert part.tolist() == H["greedy_parts"] and task.tolist() == H["greedy_task_order"]
        assert st_["loads"] == H["loads"] and st_["cost"] == H["cost"]
    for name in ("multilevel_refine5.json", "multilevel_contiguity6.json"):  # refinement; contiguity
        H = json.load(open(os.path.join(golden_dir, name)))
        E = np.array(H["edges"])
        part, task, st_ = partition(E, H["n"], H["capacity"])
        assert part.tolist() == H["ep_parts"] and task.tolist() == H["ep_task_order"]
        assert st_["loads"] == H["loads"] and st_["cost"] == H["cost"]
        part, task, _ = partition(E, H["n"], H["capacity"], "ggp")
        assert part.tolist() == H["ggp_parts"] and task.tolist() == H["ggp_task_order"]


def test_partition_parity_tet_mesh():
    T = gen.tet_mesh(16, 16, 16, seed=1)
    for cap in (64, 256):
        _check_parity(T["edges"], T["n"], cap)
    _check_parity(T["edges"], T["n"], 256, "ggp")


def test_partition_parity_rmat_bipartite():
    R = gen.rmat(scale=12, n_edges=40_000, seed=2)
    g = spmv_graph(R, R["shuffle"])
    _check_parity(g["edges"], g["n"], 256)
    _check_parity(g["edges"][:8000], g["n"], 64, "greedy")
    _check_parity(g["edges"], g["n"], 256, "random")


def _library_owned_order_ok(perm_lib, own0, nown, edges, part, task):
    """The library orders a part's owned range by the next part that touches the vertex
    (vertices no later part touches first), then by first touch."""
    parts_of, first = {}, {}
    for j, e in enumerate(task.tolist()):
        for w in (int(edges[e][0]), int(edges[e][1])):
            ps = parts_of.setdefault(w, [])
            if not ps or ps[-1] != int(part[e]):
                ps.append(int(part[e]))
            first.setdefault(w, 2 * j + (w == int(edges[e][1])))
    ids = perm_lib[own0:own0 + nown].tolist()
    key = [((parts_of[w][1] if len(parts_of[w]) > 1 else -1), first[w]) for w in ids]
    return key == sorted(key)


def _check_layout(edges, n, cap, geom, kind="flux5", n_x=0, order="ep"):
    """The library's packing against the oracle's first-touch packing (Section 4.1): the same
    owned range (start, count) per part and class, the same owned and foreign vertex sets,
    the same isolated tail; inside an owned range the library's own order rule holds."""
    P = Plan(edges, n, cap, geom, order=order, kind=kind, n_x=n_x)
    part, task = P.part_of_edge()
    lay = cpack.layout(edges, n, part, task, n_x=n_x if kind == "spmv" else None)
    perm_lib, perm_ref = P.perm(), lay["perm"]
    assert sorted(perm_lib.tolist()) == list(range(n))
    L = P.layout()
    ncls = 2 if kind == "spmv" else 1
    fo, fi = L["foreign_offset"], L["foreign_ids"]
    for p, info in enumerate(lay["parts"]):
        for c in range(ncls):
            o0, no = int(L["own_begin"][p, c]), int(L["own_count"][p, c])
            assert o0 == info["own0"][c] and no == info["nown"][c]
            assert set(perm_lib[o0:o0 + no].tolist()) == set(perm_ref[o0:o0 + no].tolist())
            assert _library_owned_order_ok(perm_lib, o0, no, edges, part, task)
            s, e = fo[p * ncls + c], fo[p * ncls + c + 1]
            assert (np.diff(fi[s:e]) > 0).all()
            assert set(perm_lib[fi[s:e]].tolist()) == set(perm_ref[info["foreign"][c]].tolist())
    iso = lay["first_part"] < 0
    for lo, hi in ([(0, n_x), (n_x, n)] if kind == "spmv" else [(0, n)]):  # each class ends with its isolated ids
        n_iso = int(iso[lo:hi].sum())
        assert np.array_equal(perm_lib[hi - n_iso:hi], perm_ref[hi - n_iso:hi])
        assert (np.diff(perm_ref[hi - n_iso:hi]) > 0).all() and iso[perm_ref[hi - n_iso:hi]].all()
    stt = P.stats
    assert stt["loads"] == sum(int(L["own_count"][p].sum()) for p in range(stt["n_parts"])) + len(fi)
    assert stt["cost"] == len(fi)


def test_plan_layout_hand_derived_three_parts(golden_dir):
    """The C++ plan packs the hand-derived case of tests/golden/cpack_three_parts.json as derived
    for the library's next-consumer order (the default order at capacity 3 is exactly that case's
    partition); owned ranges and costs are those of the first-touch packing."""
    with open(os.path.join(golden_dir, "cpack_three_parts.json")) as f:
        G = json.load(f)
    E = np.array(G["edges"], dtype=np.int32)
    geom = np.tile(np.array([[1.0, 0.0, 0.0, 1.0]], dtype=np.float32), (len(E), 1))
    P = Plan(E, G["n"], G["capacity"], geom, order="input")
    part, task = P.part_of_edge()
    assert part.tolist() == G["part"] and task.tolist() == G["task"]
    assert P.perm().tolist() == G["library_perm"]
    L = P.layout()
    fo, fi = L["foreign_offset"], L["foreign_ids"]
    assert L["own_begin"][:, 0].tolist() == G["own_begin"] and L["own_count"][:, 0].tolist() == G["own_count"]
    assert [fi[fo[p]:fo[p + 1]].tolist() for p in range(len(G["own_begin"]))] == G["library_foreign"]
    st_ = P.stats
    assert (st_["loads"], st_["cost"], st_["replicated"], st_["slots"]) == (G["loads"], G["cost"], G["replicated"],
                                                                         G["slots"])


def test_layout_parity_flux():
    G = gen.grid2d(30, 20, seed=3)
    _check_layout(G["edges"], G["n"], 64, G["geom"].astype(np.float32))
    _check_layout(G["edges"], G["n"], 64, G["geom"].astype(np.float32), order="input")
    _check_layout(G["edges"], G["n"], 64, G["geom"].astype(np.float32), order="ggp")
    T = gen.tet_mesh(6, 5, 4, seed=3)
    _check_layout(T["edges"], T["n"], 128, T["geom"].astype(np.float32))


def test_layout_parity_spmv_and_isolated():
    R = gen.rmat(scale=10, n_edges=6000, seed=5)
    g = spmv_graph(R, R["shuffle"])
    _check_layout(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"])
    _check_layout(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"], order="input")


def test_batch_set_launch_validation():
    """The batch's workgroup size: multiples of 64 up to 256 lanes, at most 8 edges per lane;
    0 keeps the current size.  Host only (no upload)."""
    from paper_1605_02043_amd.batch import Batch

    graphs = gen.batch_graphs(4, seed=2, lo=200, hi=800)
    plans = [Plan(g["edges"], g["n"], 512, g["geom"].astype(np.float32)) for g in graphs]
    B = Batch(plans)
    assert B.info()["wg"] == 256
    for bad in (32, 96, 320, 1024):
        with pytest.raises(_lib.EpkError) as e:
            B.set_launch(bad)
        assert e.value.status == _lib.EPK_EINVAL
        assert B.info()["wg"] == 256
    B.set_launch(64)  # 512 edges = 8 per lane
    assert B.info()["wg"] == 64
    B.set_launch(0)
    assert B.info()["wg"] == 64
    B2 = Batch([Plan(g["edges"], g["n"], 576, g["geom"].astype(np.float32)) for g in graphs])
    with pytest.raises(_lib.EpkError) as e:
        B2.set_launch(64)  # 9 or more edges per lane
    assert e.value.status == _lib.EPK_EINVAL
    # one workgroup per item: needs one capacity for every graph, and is then the default
    assert B.info()["direct_ok"] == 1 and B.info()["direct"] == 1
    B.set_launch(0, 0)
    assert B.info()["direct"] == 0
    B.set_launch(0, 1)
    assert B.info()["direct"] == 1 and B.info()["wg"] == 64
    B.set_launch(256, -1)
    assert B.info()["direct"] == 1 and B.info()["wg"] == 256
    with pytest.raises(_lib.EpkError) as e:
        B.set_launch(0, 2)
    assert e.value.status == _lib.EPK_EINVAL
    B.set_launch(0, 0)
    assert B.info()["direct"] == 0
    B3 = Batch([Plan(g["edges"], g["n"], c, g["geom"].astype(np.float32)) for g, c in zip(graphs, (128, 256, 128, 256))])
    assert B3.info()["direct_ok"] == 0
    with pytest.raises(_lib.EpkError) as e:
        B3.set_launch(0, 1)
    assert e.value.status == _lib.EPK_ESTATE and B3.info()["direct"] == 0


def test_plan_handles_empty_graph():
    P = Plan(np.zeros((0, 2), np.int32), 5, 16, np.zeros((0, 4), np.float32))
    assert P.stats["n_parts"] == 0 and P.stats["loads"] == 0
    assert sorted(P.perm().tolist()) == list(range(5))


def test_slot_layout_choice_and_bytes():
    """Meshes keep the part-major workspace; SpMV takes the vertex-major one while its y
    partials number at most one per eight edges (hub-split EP on R-MAT), part-major above
    (uniform EP on R-MAT, whose cut falls on the rows).
    Vertex-major: the part kernel reads one slot index per foreign entry (4 C bytes).
    Part-major: the reduction reads a 16-byte record per replicated vertex in place of
    its id and offsets (4 R + 4 (R + 1)); mesh vertices never have more than the
    record's three slots, so no slot list is read."""
    T = gen.tet_mesh(8, 8, 8, seed=0)
    P = Plan(T["edges"], T["n"], 128, T["geom"].astype(np.float32))  # two launches (the default)
    st = P.stats
    R, C = st["replicated"], st["cost"]
    a = P.info()
    assert a["vertex_major"] == 0
    P.set_slot_layout(1)
    b = P.info()
    assert b["vertex_major"] == 1 and b["bytes_fwd_kernel"] - a["bytes_fwd_kernel"] == 4 * C
    assert a["bytes_fwd"] - b["bytes_fwd"] == (16 * R - 4 * R - 4 * (R + 1)) - 4 * C
    # the slot indices (one int32 per foreign vertex of the largest part) take LDS only when vertex-major
    for key in ("lds_fwd", "lds_bwd"):
        assert b[key] - a[key] in range(4 * a["max_nf"], 4 * a["max_nf"] + 16)
    assert b["lds_pipe_bwd"] - a["lds_pipe_bwd"] in range(8 * a["max_nf"], 8 * a["max_nf"] + 16)
    P.set_slot_layout(0)
    assert P.info() == a
    with pytest.raises(_lib.EpkError):
        P.set_slot_layout(2)
    R = gen.rmat(scale=12, n_edges=60_000, seed=1)
    g = spmv_graph(R, R["shuffle"])
    m = len(g["edges"])
    seen = set()
    for kw in ({}, {"class_weight": (1, 4), "hub_degree": 16}):
        S = Plan(g["edges"], g["n"], 256, g["w"], kind="spmv", n_x=g["n_x"], **kw)
        fo = S.layout()["foreign_offset"]
        s_y = int(sum(fo[2 * p + 2] - fo[2 * p + 1] for p in range(S.stats["n_parts"])))
        vm = S.info()["vertex_major"]
        assert vm == int(8 * s_y <= m), (kw, s_y, m)
        seen.add(vm)
        S.set_slot_layout(1 - vm)
        S.set_slot_layout(-1)
        assert S.info()["vertex_major"] == vm
    assert seen == {0, 1}  # both rules' sides are exercised


def test_plan_from_caller_partition():
    """A plan built from a caller's partition equals the library's own plan for the same
    partition (layout and stats), and a part holding more edges than the capacity is refused
    before anything is packed (each part's records fill one block of cap slots)."""
    T = gen.tet_mesh(6, 6, 6, seed=3)
    E, n, geom = T["edges"], T["n"], T["geom"].astype(np.float32)
    P = Plan(E, n, 64, geom)
    part, task = P.part_of_edge()
    Q = Plan.from_partition(E, n, 64, geom, part, task, n_parts=P.stats["n_parts"])
    for key in ("n_parts", "loads", "cost", "replicated", "slots", "aux_cut", "max_part_edges"):
        assert Q.stats[key] == P.stats[key], key
    a, b = P.layout(), Q.layout()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(P.perm(), Q.perm())
    assert P.info() == Q.info()
    # default task order: ascending edge id inside a part (the EP order's own rule)
    R = Plan.from_partition(E, n, 64, geom, part)
    assert np.array_equal(R.part_of_edge()[1], task)
    # a part above the capacity: 65 edges in part 0
    over = part.copy()
    moved = np.flatnonzero(part == 1)[: 65 - int((part == 0).sum())]
    over[moved] = 0
    assert (over == 0).sum() == 65
    with pytest.raises(_lib.EpkError) as e:
        Plan.from_partition(E, n, 64, geom, over, n_parts=P.stats["n_parts"])
    assert e.value.status == _lib.EPK_ERANGE
    # the same partition fits a capacity of 65
    Plan.from_partition(E, n, 65, geom, over, n_parts=P.stats["n_parts"])
    with pytest.raises(_lib.EpkError) as e:  # an entry outside [0, n_parts)
        Plan.from_partition(E, n, 64, geom, part, n_parts=int(part.max()))
    assert e.value.status == _lib.EPK_EINVAL
    bad = task.copy()
    bad[[0, -1]] = bad[[-1, 0]]  # parts out of order
    with pytest.raises(_lib.EpkError) as e:
        Plan.from_partition(E, n, 64, geom, part, bad)
    assert e.value.status == _lib.EPK_EINVAL
    bad = task.copy()
    bad[1] = bad[0]  # not a permutation
    with pytest.raises(_lib.EpkError) as e:
        Plan.from_partition(E, n, 64, geom, part, bad)
    assert e.value.status == _lib.EPK_EINVAL


def test_binding_checks_device_buffers():
    """The binding refuses buffers the kernels would read or write out of bounds (wrong
    dtype, shape, row count, layout or device) before any library call, for Plan and Batch
    inputs and outputs alike.  Run on CPU tensors with the device set by hand: nothing
    here reaches the library's device entry points."""
    import torch

    from paper_1605_02043_amd.batch import Batch

    T = gen.tet_mesh(4, 4, 4, seed=0)
    P = Plan(T["edges"], T["n"], 64, T["geom"].astype(np.float32))
    n = T["n"]
    good = torch.zeros(n, 5)
    with pytest.raises(ValueError, match="not uploaded"):
        P.forward(good)
    P.device = torch.device("cpu")
    bad = [torch.zeros(n, 5, dtype=torch.float64), torch.zeros(n - 1, 5), torch.zeros(n, 4),
           torch.zeros(5, n).t(), torch.zeros(n * 5), np.zeros((n, 5), np.float32)]
    for b in bad:
        with pytest.raises(ValueError):
            P.forward(b)
        with pytest.raises(ValueError):
            P.forward(good, out=b)
        with pytest.raises(ValueError):
            P.backward(good, b)
        with pytest.raises(ValueError):
            P.backward(good, good, out=b)
    graphs = gen.batch_graphs(3, seed=1, lo=200, hi=600)
    B = Batch([Plan(g["edges"], g["n"], 128, g["geom"].astype(np.float32)) for g in graphs])
    good = torch.zeros(B.n, 5)
    with pytest.raises(ValueError, match="not uploaded"):
        B.forward(good)
    B.device = torch.device("cpu")
    for b in (torch.zeros(B.n - 1, 5), torch.zeros(B.n, 5, dtype=torch.float16), torch.zeros(5, B.n).t(),
              torch.zeros(graphs[0]["n"], 5)):
        with pytest.raises(ValueError):
            B.forward(b)
        with pytest.raises(ValueError):
            B.forward(good, out=b)
        with pytest.raises(ValueError):
            B.backward(good, b)
        with pytest.raises(ValueError):
            B.backward(b, good)
        with pytest.raises(ValueError):
            B.backward(good, good, out=b)


def test_forward_scratch_refuses_large_workspace():
    """epk_forward_scratch keeps the partials in a fixed 16 MiB array: a plan needing more is
    refused (EPK_ERANGE) before anything touches a device; a plan that fits but was never
    uploaded gets EPK_ESTATE."""
    lib = _lib.lib
    rng = np.random.default_rng(0)
    n, m = 300_000, 600_000
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    E = np.stack([u, v], 1).astype(np.int32)
    P = Plan(E, n, 256, np.tile(np.float32([[1, 0, 0, 1]]), (m, 1)), order="input")
    assert P.device_bytes()[1] > 16 << 20
    assert lib.epk_forward_scratch(P._h, None, None, C.c_float(0.0), None, None) == _lib.EPK_ERANGE
    assert b"16 MiB" in lib.epk_last_error()
    Q = Plan(np.array([[0, 1], [1, 2]]), 3, 4, np.zeros((2, 4), np.float32))
    assert lib.epk_forward_scratch(Q._h, None, None, C.c_float(0.0), None, None) == _lib.EPK_ESTATE
    S = Plan(np.array([[0, 2]]), 3, 4, np.ones(1, np.float32), kind="spmv", n_x=1)
    assert lib.epk_forward_scratch(S._h, None, None, C.c_float(0.0), None, None) == _lib.EPK_ESTATE


def _signals(P):
    """Signal records of the single-launch reduction, recounted from the plan's layout: each part
    signals the owner of every foreign vertex, and itself if a later part uses one of its vertices."""
    L = P.layout()
    k = P.stats["n_parts"]
    ob, oc, fo, fi = L["own_begin"][:, 0], L["own_count"][:, 0], L["foreign_offset"], L["foreign_ids"]
    owner = np.full(P.n, -1)
    for q in range(k):
        owner[ob[q]:ob[q] + oc[q]] = q
    shared = np.zeros(P.n, bool)
    shared[fi] = True
    sig = [set(owner[fi[fo[p]:fo[p + 1]]].tolist()) | ({p} if shared[ob[p]:ob[p] + oc[p]].any() else set())
           for p in range(k)]
    return sig


def test_single_launch_reduction_accounting_and_switch():
    """FLUX5 mesh plans can sum their replicated vertices inside the part kernel (off by
    default).  Its bytes are the two launches' plus 24 per signal (a 16-byte record, a 4-byte
    counter read and written); switching it off restores the two-launch figures; the
    vertex-major layout, the pipelined and the cache-only launches keep two launches; SpMV
    plans cannot switch it on."""
    T = gen.tet_mesh(8, 8, 8, seed=0)
    P = Plan(T["edges"], T["n"], 128, T["geom"].astype(np.float32))
    assert P.info()["fused"] == 0
    P.set_fused(1)
    a = P.info()
    assert a["fused"] == 1
    n_sig = sum(len(s) for s in _signals(P))
    P.set_fused(0)
    b = P.info()
    assert b["fused"] == 0
    red_f = b["bytes_fwd"] - b["bytes_fwd_kernel"]
    red_b = b["bytes_bwd"] - b["bytes_bwd_kernel"]
    assert a["bytes_fwd_kernel"] == b["bytes_fwd_kernel"] + red_f + 24 * n_sig == a["bytes_fwd"]
    assert a["bytes_bwd_kernel"] == b["bytes_bwd_kernel"] + red_b + 24 * n_sig == a["bytes_bwd"]
    P.set_fused(1)
    assert P.info() == a
    P.set_slot_layout(1)
    assert P.info()["fused"] == 0
    P.set_slot_layout(0)
    assert P.info()["fused"] == 1
    P.set_staging(0)
    assert P.info()["fused"] == 0
    P.set_staging(1)
    assert P.info()["fused"] == 1
    with pytest.raises(_lib.EpkError):
        P.set_fused(2)
    R = gen.rmat(scale=10, n_edges=6000, seed=5)
    g = spmv_graph(R, R["shuffle"])
    S = Plan(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"])
    assert S.info()["fused"] == 0
    with pytest.raises(_lib.EpkError) as e:
        S.set_fused(1)
    assert e.value.status == _lib.EPK_ESTATE
    S.set_fused(0)


def test_weighted_partition_parity_and_errors():
    """The library's weighted EP partition equals the oracle's bit for bit (random bipartite
    graphs, several weights; the hand-derived K2,2 case), {1, 1} equals the unweighted call, and
    bad weights or weights on other orders are refused."""
    from oracle import multilevel

    K22 = np.array([[0, 2], [0, 3], [1, 2], [1, 3]], dtype=np.int32)
    part, task, _ = partition(K22, 4, 2, "ep", class_weight=(1, 4), n_x=2)
    assert part.tolist() == [0, 1, 0, 1] and task.tolist() == [0, 2, 1, 3]
    rng = np.random.default_rng(77)
    for trial in range(30):
        n_x, n_y = int(rng.integers(2, 60)), int(rng.integers(2, 60))
        m = int(rng.integers(1, 700))
        cap = int(rng.integers(1, 48))
        wx, wy = int(rng.integers(1, 5)), int(rng.integers(1, 9))
        E = np.stack([rng.integers(0, n_x, m), n_x + rng.integers(0, n_y, m)], 1).astype(np.int32)
        p1, t1, st1 = partition(E, n_x + n_y, cap, "ep", class_weight=(wx, wy), n_x=n_x)
        p2, t2, _ = multilevel.partition(E, n_x + n_y, cap, class_weight=(wx, wy), n_x=n_x)
        assert np.array_equal(p1, p2) and np.array_equal(t1, t2), (trial, wx, wy)
        assert st1["max_part_edges"] <= cap
    pu, tu, _ = partition(E, n_x + n_y, cap, "ep")
    pw, tw, _ = partition(E, n_x + n_y, cap, "ep", class_weight=(1, 1), n_x=n_x)
    assert np.array_equal(pu, pw) and np.array_equal(tu, tw)
    for bad in ((0, 1), (1, 65)):
        with pytest.raises(_lib.EpkError) as e:
            partition(E, n_x + n_y, cap, "ep", class_weight=bad, n_x=n_x)
        assert e.value.status == _lib.EPK_EINVAL
    with pytest.raises(_lib.EpkError) as e:
        partition(E, n_x + n_y, cap, "ggp", class_weight=(1, 4), n_x=n_x)
    assert e.value.status == _lib.EPK_EINVAL
    partition(E, n_x + n_y, cap, "input", class_weight=(1, 1), n_x=n_x)
    g = spmv_graph(gen.rmat(scale=9, n_edges=3000, seed=4), np.arange(3000))
    P = Plan(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"], class_weight=(1, 4))
    p3, t3 = P.part_of_edge()
    p4, t4 = multilevel.partition(g["edges"], g["n"], 128, class_weight=(1, 4), n_x=g["n_x"])[:2]
    assert np.array_equal(p3, p4) and np.array_equal(t3, t4)


def test_hub_partition_parity_and_errors():
    """The library's hub split equals the oracle's bit for bit: the hand-derived cases, random
    power-law bipartite graphs with and without class weights, a small R-MAT, one-class graphs;
    the plan built with it carries the same partition; bad arguments are refused."""
    from oracle import hub

    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hub_split7.json")))
    for c in G["cases"]:
        p, t, st_ = partition(np.array(c["edges"]), c["n"], c["cap"], "ep", None, c["n_x"], c["hub_degree"])
        assert p.tolist() == c["part"] and t.tolist() == c["task"] and st_["n_parts"] == c["n_parts"]
    rng = np.random.default_rng(5)
    for trial in range(30):
        n_x, n_y = int(rng.integers(2, 50)), int(rng.integers(2, 50))
        m = int(rng.integers(1, 800))
        cap = int(rng.integers(1, 48))
        hd = int(rng.integers(1, 40))
        cw = None if trial % 2 else (1, int(rng.integers(1, 9)))
        py = 1.0 / np.arange(1, n_y + 1) ** 1.2
        E = np.stack([rng.integers(0, n_x, m), n_x + rng.choice(n_y, size=m, p=py / py.sum())], 1).astype(np.int32)
        p1, t1, st1 = partition(E, n_x + n_y, cap, "ep", cw, n_x, hd)
        p2, t2, k2 = hub.partition(E, n_x + n_y, cap, hd, cw, n_x)
        assert np.array_equal(p1, p2) and np.array_equal(t1, t2) and st1["n_parts"] == k2, trial
        assert st1["max_part_edges"] <= cap
        c = cost.partition_cost(E, n_x + n_y, p2, k2)
        assert st1["loads"] == c["loads"] and st1["cost"] == c["cost"]
    for trial in range(10):  # one class: keys by degree
        n, m = int(rng.integers(3, 40)), int(rng.integers(1, 300))
        E = rng.integers(0, n, size=(m, 2)).astype(np.int32)
        E = E[E[:, 0] != E[:, 1]]
        cap, hd = int(rng.integers(1, 30)), int(rng.integers(1, 12))
        p1, t1, _ = partition(E, n, cap, "ep", None, 0, hd)
        p2, t2, _ = hub.partition(E, n, cap, hd, None, 0)
        assert np.array_equal(p1, p2) and np.array_equal(t1, t2), trial
    g = spmv_graph(gen.rmat(scale=10, n_edges=8000, seed=6), np.arange(8000))
    P = Plan(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"], class_weight=(1, 4), hub_degree=16)
    p3, t3 = P.part_of_edge()
    p4, t4, _ = hub.partition(g["edges"], g["n"], 128, 16, (1, 4), g["n_x"])
    assert np.array_equal(p3, p4) and np.array_equal(t3, t4)
    gs, keep = make_graph(E, n, None, 0)
    part = np.empty(len(E), np.int32)
    assert _lib.lib.epk_partition_hub(C.byref(gs), 4, None, 0, _lib.i32p(part), None, None) == _lib.EPK_EINVAL
    with pytest.raises(ValueError):
        partition(E, n, 4, "ggp", None, 0, 3)
    with pytest.raises(ValueError):
        Plan(g["edges"], g["n"], 128, g["w"], kind="spmv", n_x=g["n_x"], order="input", hub_degree=4)

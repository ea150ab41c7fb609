"""The single-launch reduction (an option, off by default): the part kernel also
sums the replicated vertices (the workgroup completing a part's partials sums
them), and must give bitwise the results of the two-launch path, on every task
order, workgroup size and launch after launch (its counters return to zero),
eagerly and in captured HIP-graph replays; and its results match the FP64
oracle.

Cases include parts that signal more parts than the workgroup has lanes (the
default and random orders), untouched vertices, 2D and 3D geometry, and the
full 1M-cell mesh."""

import numpy as np
import pytest

import gen
from oracle import flux
from tests.gpu_util import assert_close, pack_rows, say, unpack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02043_amd import Plan  # noqa: F401  (fails loudly without libepk.so)


def _with_isolated(G, extra):
    """The graph with `extra` vertices no edge touches (ids interleaved with the others)."""
    n = G["n"] + extra
    ids = np.random.default_rng(11).permutation(n)[: G["n"]]
    E = ids[np.asarray(G["edges"])]
    u, v = np.minimum(E[:, 0], E[:, 1]), np.maximum(E[:, 0], E[:, 1])
    g = np.asarray(G["geom"]).copy()
    flip = E[:, 0] > E[:, 1]  # keep the normal pointing from u to v
    g[flip, :3 if g.shape[1] == 4 else 2] *= -1
    return {"n": n, "edges": np.stack([u, v], 1).astype(np.int32), "geom": g}


def _run(P, qd, gd, dt):
    r, qn = P.forward(qd, dt)
    g = P.backward(qd, gd)
    torch.cuda.synchronize()
    return r.clone(), qn.clone(), g.clone()


CASES = [("grid64", "ep", 256, 0), ("tet32", "ep", 256, 0), ("tet32", "input", 256, 0), ("tet32", "random", 256, 0),
         ("tet32", "ep", 256, 64), ("tet32", "input", 128, 64), ("iso", "ep", 64, 0)]


@pytest.mark.parametrize("name,order,cap,wg", CASES)
def test_single_launch_equals_two_launches(name, order, cap, wg):
    from paper_1605_02043_amd import Plan

    G = _with_isolated(gen.tet_mesh(10, 9, 8, seed=2), 300) if name == "iso" else gen.workload(name, seed=0)
    say(f"case fused {name} order={order} cap={cap} wg={wg or 'default'} n={G['n']} m={len(G['edges'])}")
    P = Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32), order=order)
    if wg:
        P.set_launch(wg)
    P.upload("cuda")
    P.set_fused(1)
    assert P.info()["fused"] == 1
    perm = P.perm()
    q = gen.flux_state(G["n"], seed=1)
    gr = gen.workloads.grad_seed(G["n"], seed=1)
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    one = [_run(P, qd, gd, 0.05) for _ in range(3)]  # launch after launch: the counters return to zero
    P.set_fused(0)
    assert P.info()["fused"] == 0
    two = _run(P, qd, gd, 0.05)
    P.set_fused(1)
    for rep, res in enumerate(one):
        for a, b, what in zip(res, two, ("r", "q_new", "g_q")):
            assert torch.equal(a, b), f"{what} differs from the two-launch path (launch {rep})"
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    r = unpack_rows(one[0][0].cpu().numpy(), perm)
    g = unpack_rows(one[0][2].cpu().numpy(), perm)
    assert_close(f"fused/{name}/{order}/r", r, flux.forward(G["n"], G["edges"], g64, q),
                 flux.forward_abs(G["n"], G["edges"], g64, q))
    assert_close(f"fused/{name}/{order}/g_q", g, flux.backward(G["n"], G["edges"], g64, q, gr),
                 flux.backward_abs(G["n"], G["edges"], g64, q, gr))
    if name == "iso":
        untouched = np.setdiff1d(np.arange(G["n"]), np.asarray(G["edges"]).ravel())
        assert (r[untouched] == 0).all() and (g[untouched] == 0).all()


def test_single_launch_graph_replays_and_two_plans():
    """Forward then adjoint (upstream gradient r) of two plans captured in one HIP graph and
    replayed several times, with eager launches of both plans between the replays: every
    replay equals the eager two-launch results bit for bit."""
    from paper_1605_02043_amd import Plan

    plans, ins, refs = [], [], []
    for name, order in (("tet32", "ep"), ("grid64", "input")):
        G = gen.workload(name, seed=0)
        P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32), order=order).upload("cuda")
        qd = torch.from_numpy(gen.flux_state(G["n"], seed=2)[P.perm()]).cuda()
        assert P.info()["fused"] == 0  # the default: two launches
        P.set_fused(0)
        r0 = P.forward(qd)
        g0 = P.backward(qd, r0)
        torch.cuda.synchronize()
        P.set_fused(1)
        plans.append(P)
        ins.append(qd)
        refs.append((r0.clone(), g0.clone()))
    outs = [(torch.empty_like(qd), torch.empty_like(qd)) for qd in ins]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for P, qd, (r, g) in zip(plans, ins, outs):
            P.forward(qd, out=r)
            P.backward(qd, r, out=g)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for P, qd, (r, g) in zip(plans, ins, outs):
            P.forward(qd, out=r)
            P.backward(qd, r, out=g)
    for rep in range(4):
        say(f"  replay {rep}")
        for r, g in outs:
            r.fill_(float("nan"))
            g.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        for (r, g), (r0, g0) in zip(outs, refs):
            assert torch.equal(r, r0) and torch.equal(g, g0)
        for P, qd in zip(plans, ins):  # eager work between replays
            P.backward(qd, P.forward(qd))
        torch.cuda.synchronize()


def test_single_launch_tet55_full_size():
    from paper_1605_02043_amd import Plan

    G = gen.workload("tet55", seed=0)
    say(f"case fused tet55 n={G['n']} m={len(G['edges'])}")
    P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32)).upload("cuda")
    P.set_fused(1)
    assert P.info()["fused"] == 1
    perm = P.perm()
    q = gen.flux_state(G["n"], seed=0)
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    r1 = P.forward(qd)
    g1 = P.backward(qd, r1)
    torch.cuda.synchronize()
    P.set_fused(0)
    r2 = P.forward(qd)
    g2 = P.backward(qd, r2)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(g1, g2)
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    ref = flux.forward(G["n"], G["edges"], g64, q)
    A = flux.forward_abs(G["n"], G["edges"], g64, q)
    assert_close("fused/tet55/r", unpack_rows(r1.cpu().numpy(), perm), ref, A)
    gref = flux.backward(G["n"], G["edges"], g64, q, unpack_rows(r1.cpu().numpy(), perm).astype(np.float64))
    gA = flux.backward_abs(G["n"], G["edges"], g64, q, np.abs(ref) + A)
    assert_close("fused/tet55/g_q", unpack_rows(g1.cpu().numpy(), perm), gref, gA)

"""Batched persistent launch: results equal the per-graph oracle, replays of a
captured HIP graph equal the eager run, and the autotuner returns valid caps."""

import numpy as np
import pytest

import gen
from oracle import flux
from tests.gpu_util import assert_close, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _build(graphs, caps):
    from paper_1605_02043_amd import Plan
    from paper_1605_02043_amd.batch import Batch

    plans = [Plan(g["edges"], g["n"], int(c), g["geom"].astype(np.float32)) for g, c in zip(graphs, caps)]
    B = Batch(plans).upload("cuda")
    return plans, B


def _pack_all(graphs, plans, arrs):
    return np.concatenate([a[p.perm()] for a, p in zip(arrs, plans)]).astype(np.float32)


def _unpack_all(graphs, plans, B, packed):
    out = []
    for i, p in enumerate(plans):
        blk = packed[B.offsets[i]:B.offsets[i + 1]]
        o = np.empty_like(blk)
        o[p.perm()] = blk
        out.append(o)
    return out


def _check(graphs, plans, B, tag):
    qs = [gen.flux_state(g["n"], seed=i) for i, g in enumerate(graphs)]
    grs = [gen.workloads.grad_seed(g["n"], seed=i) for i, g in enumerate(graphs)]
    qd = torch.from_numpy(_pack_all(graphs, plans, qs)).cuda()
    gd = torch.from_numpy(_pack_all(graphs, plans, grs)).cuda()
    r = _unpack_all(graphs, plans, B, B.forward(qd).cpu().numpy())
    gq = _unpack_all(graphs, plans, B, B.backward(qd, gd).cpu().numpy())
    for i, g in enumerate(graphs):
        geo = g["geom"].astype(np.float32).astype(np.float64)
        assert_close(f"{tag}/g{i}/r", r[i], flux.forward(g["n"], g["edges"], geo, qs[i]),
                     flux.forward_abs(g["n"], g["edges"], geo, qs[i]))
        assert_close(f"{tag}/g{i}/g_q", gq[i], flux.backward(g["n"], g["edges"], geo, qs[i], grs[i]),
                     flux.backward_abs(g["n"], g["edges"], geo, qs[i], grs[i]))
    return qd, gd


def test_batch_small_mixed_caps():
    graphs = gen.batch_graphs(12, seed=3, lo=200, hi=4000)
    caps = [64, 128, 256, 512] * 3
    say("case batch12 mixed caps")
    plans, B = _build(graphs, caps)
    say(f"  info {B.info()}")
    _check(graphs, plans, B, "batch12")


def test_batch_launch_shapes_bitwise():
    """The launch shape (workgroup size; pipelined persistent or one workgroup per item) changes
    lanes per edge and the order parts run in, never a result bit."""
    graphs = gen.batch_graphs(12, seed=5, lo=200, hi=4000)
    for cap, shapes in ((256, ((128, 0), (256, 1), (128, 1))), (128, ((64, 0), (256, 0), (128, 1), (64, 1)))):
        say(f"case batch12 cap {cap} launch shapes {shapes}")
        plans, B = _build(graphs, [cap] * len(graphs))
        qd, gd = _check(graphs, plans, B, f"batch12/cap{cap}")
        r0, g0 = B.forward(qd).clone(), B.backward(qd, gd).clone()
        for wg, direct in shapes:
            B.set_launch(wg, direct)
            say(f"  wg {wg} direct {direct}: {B.info()}")
            assert B.info()["wg"] == wg and B.info()["direct"] == direct
            assert torch.equal(B.forward(qd), r0) and torch.equal(B.backward(qd, gd), g0)


def _unit_geom(m, rng):
    nrm = rng.standard_normal((m, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return np.concatenate([nrm, rng.uniform(0.5, 2.0, (m, 1))], axis=1).astype(np.float32)


def test_batch_edge_cases_both_launch_kinds():
    """Empty graphs, a single edge, isolated vertices, a hub and parts with more foreign ids
    than lanes, in one batch: both launch kinds against the oracle and bitwise equal."""
    rng = np.random.default_rng(11)
    graphs = []
    graphs.append({"edges": np.zeros((0, 2), np.int64), "n": 7})
    graphs.append({"edges": np.array([[3, 1]]), "n": 6})
    n, m = 50, 203
    u = rng.integers(0, n, m)
    graphs.append({"edges": np.stack([u, (u + 1 + rng.integers(0, n - 1, m)) % n], 1), "n": n + 5})
    graphs.append({"edges": np.zeros((0, 2), np.int64), "n": 1})
    graphs.append({"edges": np.stack([np.zeros(299, int), np.arange(1, 300)], 1), "n": 300})
    n, m = 1200, 5000
    u = rng.integers(0, n, m)
    graphs.append({"edges": np.stack([u, (u + 1 + rng.integers(0, n - 1, m)) % n], 1), "n": n})
    for g in graphs:
        g["geom"] = _unit_geom(len(g["edges"]), rng)
    for cap in (16, 512):
        say(f"case batch edge cases cap {cap}")
        plans, B = _build(graphs, [cap] * len(graphs))
        assert B.info()["direct_ok"] == 1
        outs = []
        for direct in (1, 0):
            B.set_launch(0, direct)
            say(f"  direct {direct}: {B.info()}")
            qd, gd = _check(graphs, plans, B, f"edge/cap{cap}/direct{direct}")
            outs.append((B.forward(qd).clone(), B.backward(qd, gd).clone()))
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_batch_hubs_vertex_major_both_launch_kinds():
    """Hub-heavy graphs put the batch in the vertex-major workspace (slots scattered through
    per-entry slot indices), and at capacity 4 the largest hub has more partials than one
    reduction thread takes: both launch kinds against the oracle and bitwise equal."""
    rng = np.random.default_rng(13)
    graphs = []
    for leaves in (299, 150, 400):
        graphs.append({"edges": np.stack([np.zeros(leaves, int), np.arange(1, leaves + 1)], 1), "n": leaves + 1})
    n, m = 40, 120
    u = rng.integers(0, n, m)
    graphs.append({"edges": np.stack([u, (u + 1 + rng.integers(0, n - 1, m)) % n], 1), "n": n})
    for g in graphs:
        g["geom"] = _unit_geom(len(g["edges"]), rng)
    for cap in (4, 16):
        say(f"case batch hubs cap {cap}")
        plans, B = _build(graphs, [cap] * len(graphs))
        outs = []
        for direct in (1, 0):
            B.set_launch(0, direct)
            say(f"  direct {direct}: {B.info()}")
            qd, gd = _check(graphs, plans, B, f"hubs/cap{cap}/direct{direct}")
            outs.append((B.forward(qd).clone(), B.backward(qd, gd).clone()))
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_batch256_and_graph_replay():
    graphs = gen.batch_graphs(256, seed=0)
    caps = [256] * len(graphs)
    say(f"case batch256 total n={sum(g['n'] for g in graphs)} m={sum(len(g['edges']) for g in graphs)}")
    plans, B = _build(graphs, caps)
    say(f"  info {B.info()}")
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(len(graphs), 16, replace=False).tolist())
    q = torch.from_numpy(_pack_all(graphs, plans, [gen.flux_state(g["n"], seed=i) for i, g in enumerate(graphs)])).cuda()
    gr = torch.from_numpy(_pack_all(graphs, plans, [gen.workloads.grad_seed(g["n"], seed=i) for i, g in enumerate(graphs)])).cuda()
    r_eager = B.forward(q).clone()
    g_eager = B.backward(q, gr).clone()
    rr = _unpack_all(graphs, plans, B, r_eager.cpu().numpy())
    for i in pick:
        g = graphs[i]
        qi = gen.flux_state(g["n"], seed=i)
        geo = g["geom"].astype(np.float32).astype(np.float64)
        assert_close(f"batch256/g{i}/r", rr[i], flux.forward(g["n"], g["edges"], geo, qi),
                     flux.forward_abs(g["n"], g["edges"], geo, qi))
    # capture forward + adjoint into one graph, replay several times with eager work between
    r_out = torch.empty_like(q)
    g_out = torch.empty_like(q)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.forward(q, out=r_out)
        B.backward(q, gr, out=g_out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.forward(q, out=r_out)
        B.backward(q, gr, out=g_out)
    for rep in range(4):
        say(f"  replay {rep}")
        r_out.fill_(float("nan"))
        g_out.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r_out, r_eager) and torch.equal(g_out, g_eager)
        B.forward(q)  # eager work between replays
        torch.cuda.synchronize()


def test_plan_graph_replay_matches_eager():
    from paper_1605_02043_amd import Plan

    G = gen.workload("tet32", seed=0)
    say("case plan graph replay")
    P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32)).upload("cuda")
    q = torch.from_numpy(gen.flux_state(G["n"], seed=0)[P.perm()]).cuda()
    r_eager, qn_eager = P.forward(q, dt=0.1)
    g_eager = P.backward(q, r_eager)
    r = torch.empty_like(q)
    g = torch.empty_like(q)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P.forward(q, out=r)
        P.backward(q, r, out=g)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.forward(q, out=r)
        P.backward(q, r, out=g)
    for rep in range(3):
        r.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r, r_eager) and torch.equal(g, g_eager)
        P.forward(q, dt=0.1)
        torch.cuda.synchronize()


def test_autotune_picks_listed_caps(tmp_path):
    from paper_1605_02043_amd.batch import autotune

    graphs = gen.batch_graphs(20, seed=1, lo=1024, hi=16384)
    say("case autotune")
    cache = str(tmp_path / "tune.txt")
    caps, wgs, directs = autotune(graphs, caps=(64, 128, 256, 512), cache_path=cache)
    say(f"  chose cap {caps[0]} wg {wgs[0]} direct {directs[0]}")
    assert set(caps.tolist()) <= {64, 128, 256, 512}
    assert len(set(caps.tolist())) == 1 and len(set(wgs.tolist())) == 1 and len(set(directs.tolist())) == 1
    assert wgs[0] in (64, 128, 256) and 2 * wgs[0] >= caps[0] and directs[0] in (0, 1)
    caps2, wgs2, directs2 = autotune(graphs, caps=(64, 128, 256, 512), cache_path=cache)  # from the cache
    assert np.array_equal(caps, caps2) and np.array_equal(wgs, wgs2) and np.array_equal(directs, directs2)
    plans, B = _build(graphs, caps)
    B.set_launch(int(wgs[0]), int(directs[0]))
    _check(graphs, plans, B, "tuned")

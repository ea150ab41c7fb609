"""The pipelined persistent launch (epk_plan_set_pipeline) against the
one-part-per-workgroup launch (bitwise) and against the FP64 oracle.

The pipelined kernels run the same per-part code in the same order, so their
results must equal the direct kernels' bit for bit, for every grid size
(several parts per workgroup, wrapping the pipeline many times), mapping and
edges-per-thread setting."""

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
    from paper_1605_02043_amd import Plan  # noqa: F401


def _plan(G, cap, order="ep"):
    from paper_1605_02043_amd import Plan

    return Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32), order=order).upload("cuda")


def _geom32(G):
    return G["geom"].astype(np.float32).astype(np.float64)


def _run(P, qd, gd, dt):
    r, qn = P.forward(qd, dt)
    g = P.backward(qd, gd)
    torch.cuda.synchronize()
    return r.cpu(), qn.cpu(), g.cpu()


@pytest.mark.parametrize("cap,wg", [(256, 256), (64, 64), (512, 256), (256, 128), (100, 64)])
def test_pipe_bitwise_equals_direct(cap, wg):
    G = gen.workload("tet32", seed=1)
    q = gen.flux_state(G["n"], seed=1)
    gr = gen.workloads.grad_seed(G["n"], seed=1)
    P = _plan(G, cap)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    for sw in (1, 0):
        P.set_launch(wg, sw)
        say(f"case pipe cap={cap} wg={wg} swizzle={sw} direct")
        ref = _run(P, qd, gd, 0.01)
        for per_cu in (-1, 1, 2):
            P.set_pipeline(per_cu)
            info = P.info()
            say(f"case pipe cap={cap} wg={wg} swizzle={sw} per_cu={per_cu} grid={info['grid_pipe_fwd']}/"
                f"{info['grid_pipe_bwd']} k={info['n_parts']}")
            got = _run(P, qd, gd, 0.01)
            for a, b, nm in zip(got, ref, ("r", "q_new", "g_q")):
                assert torch.equal(a, b), f"{nm} differs (cap={cap} wg={wg} swizzle={sw} per_cu={per_cu})"


def test_pipe_oracle_tet55_full_size():
    G = gen.workload("tet55", seed=0)
    say(f"case pipe tet55 n={G['n']} m={len(G['edges'])}")
    q = gen.flux_state(G["n"], seed=0)
    g = _geom32(G)
    r64 = flux.forward(G["n"], G["edges"], g, q)
    gr = (2.0 * r64).astype(np.float32)
    P = _plan(G, 256)
    P.set_pipeline(-1)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    r = unpack_rows(P.forward(qd).cpu().numpy(), perm)
    assert_close("pipe/tet55/r", r, r64, flux.forward_abs(G["n"], G["edges"], g, q))
    gq = unpack_rows(P.backward(qd, torch.from_numpy(pack_rows(gr, perm)).cuda()).cpu().numpy(), perm)
    assert_close("pipe/tet55/g_q", gq, flux.backward(G["n"], G["edges"], g, q, gr),
                 flux.backward_abs(G["n"], G["edges"], g, q, gr))


def _small(edges, n, cap, dim, seed, order="ep", per_cu=-1):
    rng = np.random.default_rng(seed)
    edges = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    v = rng.standard_normal((len(edges), 3))
    if dim == 2:
        v = v[:, :2]
    v /= np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-12)
    geom = v if dim == 2 else np.concatenate([v, rng.uniform(0.5, 2.0, (len(edges), 1))], 1)
    G = {"edges": edges, "n": n, "geom": geom}
    q = gen.flux_state(n, seed=seed)
    gr = gen.workloads.grad_seed(n, seed=seed)
    P = _plan(G, cap, order)
    P.set_pipeline(per_cu)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    r, qn, gq = (unpack_rows(x.numpy(), perm) for x in _run(P, qd, torch.from_numpy(pack_rows(gr, perm)).cuda(), -0.5))
    g = _geom32(G)
    ref, qref = flux.forward(n, edges, g, q, dt=-0.5)
    A, qA = flux.forward_abs(n, edges, g, q, dt=-0.5)
    assert_close("pipe-edge/r", r, ref, A)
    assert_close("pipe-edge/q_new", qn, qref, qA)
    assert_close("pipe-edge/g_q", gq, flux.backward(n, edges, g, q, gr), flux.backward_abs(n, edges, g, q, gr))


def test_pipe_edge_cases():
    say("case pipe empty graph")
    _small(np.zeros((0, 2)), 7, 16, 3, 0)
    say("case pipe single edge")
    _small([[3, 1]], 6, 4, 3, 0)
    rng = np.random.default_rng(1)
    n, m = 50, 203
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    for cap in (1, 7, 64, 512):
        say(f"case pipe ragged cap={cap}")
        _small(np.stack([u, v], 1), n + 5, cap, 3, cap, per_cu=1)
    star = np.stack([np.zeros(299, int), np.arange(1, 300)], 1)
    say("case pipe hub 2D")
    _small(star, 300, 16, 2, 3)
    say("case pipe hub 3D input order")
    _small(star, 300, 16, 3, 4, order="input")
    say("case pipe heavy hub cap=2")
    _small(star, 300, 2, 2, 5)
    n, m = 1200, 5000  # capacity 512: more foreign ids and vertices per part than lanes
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    say("case pipe dense parts cap=512")
    _small(np.stack([u, v], 1), n, 512, 3, 7)


def test_pipe_grid64_2d_both_orders():
    G = gen.workload("grid64", seed=0)
    q = gen.flux_state(G["n"], seed=0)
    g = _geom32(G)
    for order in ("ep", "input"):
        say(f"case pipe grid64 order={order}")
        P = _plan(G, 256, order)
        P.set_pipeline(-1)
        perm = P.perm()
        r, qn = P.forward(torch.from_numpy(pack_rows(q, perm)).cuda(), 0.01)
        ref, qref = flux.forward(G["n"], G["edges"], g, q, dt=0.01)
        A, qA = flux.forward_abs(G["n"], G["edges"], g, q, dt=0.01)
        assert_close(f"pipe/grid64/{order}/r", unpack_rows(r.cpu().numpy(), perm), ref, A)
        assert_close(f"pipe/grid64/{order}/q_new", unpack_rows(qn.cpu().numpy(), perm), qref, qA)


def test_pipe_graph_replays_match_eager():
    G = gen.workload("tet32", seed=0)
    q = gen.flux_state(G["n"], seed=0)
    gr = gen.workloads.grad_seed(G["n"], seed=0)
    P = _plan(G, 256)
    P.set_pipeline(-1)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    r = torch.empty_like(qd)
    gq = torch.empty_like(qd)
    eager_r = P.forward(qd).clone()
    eager_g = P.backward(qd, gd).clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.forward(qd, out=r)
        P.backward(qd, gd, out=gq)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.forward(qd, out=r)
        P.backward(qd, gd, out=gq)
    for i in range(4):
        say(f"case pipe graph replay {i}")
        r.zero_()
        gq.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r, eager_r) and torch.equal(gq, eager_g)
        P.forward(qd)  # eager work between replays
        torch.cuda.synchronize()

"""Workspace layouts (epk_plan_set_slot_layout): part-major and vertex-major
partials must give bit-identical results, since the reduction adds every
vertex's partials in ascending part order under both."""

import numpy as np
import pytest

import gen
from gen.rmat import spmv_graph
from oracle import spmv
from tests.gpu_util import assert_close, pack_rows, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02043_amd import Plan  # noqa: F401


def test_flux_layouts_and_launches_bitwise():
    from paper_1605_02043_amd import Plan

    G = gen.workload("tet32", seed=0)
    q = gen.flux_state(G["n"], seed=0)
    gr = gen.workloads.grad_seed(G["n"], seed=0)
    P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32)).upload("cuda")
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    ref = None
    for layout in (0, 1):
        P.set_slot_layout(layout)
        for pipe in (0, -1):
            P.set_pipeline(pipe)
            say(f"case layout={layout} pipe={pipe}")
            r, qn = P.forward(qd, 0.01)
            g = P.backward(qd, gd)
            got = (r.cpu(), qn.cpu(), g.cpu())
            if ref is None:
                ref = got
            for a, b, nm in zip(got, ref, ("r", "q_new", "g_q")):
                assert torch.equal(a, b), f"{nm} differs at layout={layout} pipe={pipe}"


@pytest.mark.parametrize("order", ["ep", "input"])
def test_spmv_layouts_bitwise_and_oracle(order):
    from paper_1605_02043_amd import Plan

    R = gen.rmat(scale=15, n_edges=1 << 19, seed=3)
    g = spmv_graph(R, R["shuffle"])
    P = Plan(g["edges"], g["n"], 256, g["w"], order=order, kind="spmv", n_x=g["n_x"]).upload("cuda")
    perm = P.perm()
    xp = torch.from_numpy(np.ascontiguousarray(R["x"][perm[:g["n_x"]]])).cuda()
    ys = []
    for layout in (0, 1):
        say(f"case spmv layout={layout} order={order}")
        P.set_slot_layout(layout)
        ys.append(P.spmv(xp).cpu())
    assert torch.equal(ys[0], ys[1])
    out = np.empty(g["n"] - g["n_x"], dtype=np.float32)
    out[perm[g["n_x"]:] - g["n_x"]] = ys[1].numpy()
    assert_close(f"spmv-layout/{order}", out, spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"]),
                 spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"]))


@pytest.mark.parametrize("cap,wg", [(256, 256), (512, 256), (64, 64), (100, 64)])
def test_cache_only_kernels_match_staged_and_oracle(cap, wg):
    """The paper's cache-only variant (no LDS staging of states): bitwise equal across workspace
    layouts, and within the oracle tolerance of the staged kernels (the two kernels are compiled
    separately, so the compiler may contract multiply-adds differently)."""
    from oracle import flux
    from paper_1605_02043_amd import Plan
    from tests.gpu_util import unpack_rows

    G = gen.workload("tet32", seed=2)
    q = gen.flux_state(G["n"], seed=2)
    gr = gen.workloads.grad_seed(G["n"], seed=2)
    P = Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32)).upload("cuda")
    P.set_launch(wg, 1)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    out = {}
    for staged in (1, 0):
        P.set_staging(staged)
        for layout in (0, 1):
            P.set_slot_layout(layout)
            say(f"case cache-only cap={cap} wg={wg} staged={staged} layout={layout}")
            r, qn = P.forward(qd, -0.25)
            out[(staged, layout)] = (r.cpu(), qn.cpu(), P.backward(qd, gd).cpu())
    for staged in (1, 0):
        for a, b, nm in zip(out[(staged, 1)], out[(staged, 0)], ("r", "q_new", "g_q")):
            assert torch.equal(a, b), f"{nm} differs between layouts (staged={staged})"
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    ref, qref = flux.forward(G["n"], G["edges"], g64, q, dt=-0.25)
    A, qA = flux.forward_abs(G["n"], G["edges"], g64, q, dt=-0.25)
    gref = flux.backward(G["n"], G["edges"], g64, q, gr)
    gA = flux.backward_abs(G["n"], G["edges"], g64, q, gr)
    for staged in (1, 0):
        r, qn, g = (unpack_rows(x.numpy(), perm) for x in out[(staged, 0)])
        assert_close(f"cache-only/{cap}/{wg}/staged={staged}/r", r, ref, A)
        assert_close(f"cache-only/{cap}/{wg}/staged={staged}/q_new", qn, qref, qA)
        assert_close(f"cache-only/{cap}/{wg}/staged={staged}/g_q", g, gref, gA)


def test_cache_only_edge_cases_against_oracle():
    from oracle import flux
    from paper_1605_02043_amd import Plan
    from tests.gpu_util import unpack_rows

    rng = np.random.default_rng(5)
    n, m = 60, 257
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    cases = [("empty", np.zeros((0, 2), np.int64), 9, 16, 3), ("single", np.array([[4, 2]]), 7, 4, 3),
             ("ragged-1", np.stack([u, v], 1), n + 3, 1, 3), ("ragged-7", np.stack([u, v], 1), n + 3, 7, 3),
             ("hub-2d", np.stack([np.zeros(199, int), np.arange(1, 200)], 1), 200, 16, 2)]
    for name, E, nv, cap, dim in cases:
        say(f"case cache-only {name}")
        geom = rng.standard_normal((len(E), 3))[:, :dim]
        geom /= np.maximum(np.linalg.norm(geom, axis=1, keepdims=True), 1e-12)
        if dim == 3:
            geom = np.concatenate([geom, rng.uniform(0.5, 2.0, (len(E), 1))], 1)
        P = Plan(E, nv, cap, geom.astype(np.float32)).upload("cuda")
        P.set_staging(0)
        perm = P.perm()
        q = gen.flux_state(nv, seed=1)
        gr = gen.workloads.grad_seed(nv, seed=1)
        qd = torch.from_numpy(pack_rows(q, perm)).cuda()
        r, qn = P.forward(qd, 0.5)
        g = P.backward(qd, torch.from_numpy(pack_rows(gr, perm)).cuda())
        g64 = geom.astype(np.float32).astype(np.float64)
        ref, qref = flux.forward(nv, E, g64, q, dt=0.5)
        A, qA = flux.forward_abs(nv, E, g64, q, dt=0.5)
        assert_close(f"cache-only/{name}/r", unpack_rows(r.cpu().numpy(), perm), ref, A)
        assert_close(f"cache-only/{name}/q_new", unpack_rows(qn.cpu().numpy(), perm), qref, qA)
        assert_close(f"cache-only/{name}/g_q", unpack_rows(g.cpu().numpy(), perm), flux.backward(nv, E, g64, q, gr),
                     flux.backward_abs(nv, E, g64, q, gr))


def test_adaptive_flux_switches_and_matches_oracle():
    """Default order first, the partitioned plan once its background build finishes; the
    state follows the switch and the results stay those of the oracle."""
    import time

    from oracle import flux
    from paper_1605_02043_amd.adaptive import AdaptiveFlux

    G = gen.workload("tet32", seed=1)
    q0 = gen.flux_state(G["n"], seed=1)
    ad = AdaptiveFlux(G["edges"], G["n"], 256, G["geom"].astype(np.float32), min_saving=0.05)
    q = ad.pack(q0)
    t0 = time.perf_counter()
    while ad.decision is None and time.perf_counter() - t0 < 60:
        q = ad.maybe_switch(q)
        ad.forward(q)
    torch.cuda.synchronize()
    say(f"case adaptive decision={ad.decision} timings={ad.timings}")
    assert ad.decision in ("ep", "input")
    r = ad.unpack(ad.forward(q))
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    assert_close("adaptive/r", r, flux.forward(G["n"], G["edges"], g64, q0), flux.forward_abs(G["n"], G["edges"], g64, q0))
    assert np.array_equal(ad.unpack(q), q0.astype(np.float32))
    ad.close()

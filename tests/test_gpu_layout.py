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

"""GPU parity of the SpMV kernel (y_i += w_e x_j) against the FP64 oracle."""

import numpy as np
import pytest

import gen
from gen.rmat import spmv_graph
from oracle import spmv
from tests.gpu_util import assert_close, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(g, cap, order, x, class_weight=None, hub_degree=0):
    from paper_1605_02043_amd import Plan

    P = Plan(g["edges"], g["n"], cap, g["w"], order=order, kind="spmv", n_x=g["n_x"],
             class_weight=class_weight, hub_degree=hub_degree).upload("cuda")
    perm = P.perm()
    n_x = g["n_x"]
    xp = torch.from_numpy(np.ascontiguousarray(x[perm[:n_x]])).cuda()
    y = P.spmv(xp)
    torch.cuda.synchronize()
    yp = y.cpu().numpy()
    out = np.empty(g["n"] - n_x, dtype=np.float32)
    out[perm[n_x:] - n_x] = yp
    return out, P


@pytest.mark.parametrize("order", ["ep", "input"])
@pytest.mark.parametrize("cap", [256, 64, 1024])
def test_spmv_rmat_small(order, cap):
    R = gen.rmat(scale=14, n_edges=1 << 18, seed=1)
    g = spmv_graph(R, R["shuffle"])
    say(f"case spmv scale14 order={order} cap={cap}")
    y, P = _run(g, cap, order, R["x"])
    ref = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    A = spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    assert_close(f"spmv14/{order}/{cap}", y, ref, A)


@pytest.mark.parametrize("cap,hub", [(256, 0), (1024, 0), (256, 16), (1024, 64)])
def test_spmv_rmat_weighted_partition(cap, hub):
    """EP with y copies weighing 4 (the partition cuts x chains before y chains), alone and after
    the hub split (the rows above `hub` nonzeros in runs of cap): the same kernels on plans
    with few replicated y, forward and adjoint against the oracle."""
    R = gen.rmat(scale=14, n_edges=1 << 18, seed=2)
    g = spmv_graph(R, R["shuffle"])
    say(f"case spmv scale14 weighted cap={cap} hub={hub}")
    y, P = _run(g, cap, "ep", R["x"], class_weight=(1, 4), hub_degree=hub)
    ref = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    A = spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    assert_close(f"spmv14/weighted/{cap}/{hub}", y, ref, A)
    perm = P.perm()
    n_x = g["n_x"]
    gy = np.random.default_rng(3).standard_normal(g["n"] - n_x).astype(np.float32)
    gyp = torch.from_numpy(np.ascontiguousarray(gy[perm[n_x:] - n_x])).cuda()
    gx = P.spmv_adjoint(gyp)
    torch.cuda.synchronize()
    out = np.empty(n_x, dtype=np.float32)
    out[perm[:n_x]] = gx.cpu().numpy()
    gref = spmv.backward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)[0]
    gA = spmv.backward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)[0]
    assert_close(f"spmv14/weighted/{cap}/{hub}/adjoint", out, gref, gA)


def test_spmv_rmat_full_size_orders():
    R = gen.rmat(scale=20, n_edges=1 << 24, seed=0)
    say("case spmv rmat20 full size")
    orders = {
        "shuffled-ep": (R["shuffle"], "ep", None, 0),
        "shuffled-ep-hub16": (R["shuffle"], "ep", (1, 4), 16),
        "shuffled": (R["shuffle"], "input", None, 0),
        "row-sorted": (np.argsort(R["rows"], kind="stable"), "input", None, 0),
    }
    ref = A = None
    for name, (perm_e, order, cw, hub) in orders.items():
        g = spmv_graph(R, perm_e)
        if ref is None:
            ref = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
            A = spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
        say(f"case spmv rmat20 {name}")
        y, P = _run(g, 256, order, R["x"], class_weight=cw, hub_degree=hub)
        assert_close(f"spmv20/{name}", y, ref, A)
        if name == "shuffled-ep":
            st = P.stats
            say(f"  loads/edge={st['loads'] / len(g['edges']):.3f} heavy-reduced vertices present")


def test_spmv_hub_row_and_determinism():
    """One row holding half of all nonzeros: a heavy vertex in the reduction."""
    rng = np.random.default_rng(5)
    n_x, n_y, m = 4000, 300, 60_000
    rows = np.where(rng.random(m) < 0.5, 7, rng.integers(0, n_y, m))
    cols = rng.integers(0, n_x, m)
    R = {"rows": rows.astype(np.int32), "cols": cols.astype(np.int32), "w": rng.random(m, dtype=np.float32),
         "n_x": n_x, "n_y": n_y}
    x = rng.standard_normal(n_x).astype(np.float32)
    g = spmv_graph(R, rng.permutation(m))
    ref = spmv.forward(n_x, n_y, g["edges"], g["w"], x)
    A = spmv.forward_abs(n_x, n_y, g["edges"], g["w"], x)
    for order in ("ep", "input"):
        say(f"case spmv hub order={order}")
        y1, P = _run(g, 128, order, x)
        y2, _ = _run(g, 128, order, x)
        assert np.array_equal(y1, y2)
        assert_close(f"spmv-hub/{order}", y1, ref, A)


@pytest.mark.parametrize("order,cap", [("ep", 256), ("input", 256), ("ep", 64), ("ep", 1024)])
def test_spmv_adjoint_against_oracle(order, cap):
    """g_x = A^T g_y and the weight gradient, through the C ABI, against the FP64 oracle."""
    from paper_1605_02043_amd import Plan

    R = gen.rmat(scale=14, n_edges=1 << 18, seed=5)
    g = spmv_graph(R, R["shuffle"])
    say(f"case spmv adjoint order={order} cap={cap}")
    P = Plan(g["edges"], g["n"], cap, g["w"], order=order, kind="spmv", n_x=g["n_x"]).upload("cuda")
    perm = P.perm()
    n_x = g["n_x"]
    rng = np.random.default_rng(1)
    gy = rng.standard_normal(R["n_y"]).astype(np.float32)
    xp = torch.from_numpy(np.ascontiguousarray(R["x"][perm[:n_x]])).cuda()
    gyp = torch.from_numpy(np.ascontiguousarray(gy[perm[n_x:] - n_x])).cuda()
    g_x, g_w = P.spmv_adjoint(gyp, xp, weights_grad=True)
    torch.cuda.synchronize()
    gx = np.empty(n_x, dtype=np.float32)
    gx[perm[:n_x]] = g_x.cpu().numpy()
    ref_x, ref_w = spmv.backward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)
    abs_x, abs_w = spmv.backward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)
    assert_close(f"spmv-adj/{order}/{cap}/g_x", gx, ref_x, abs_x)
    assert_close(f"spmv-adj/{order}/{cap}/g_w", g_w.cpu().numpy(), ref_w, abs_w)
    assert torch.equal(P.spmv_adjoint(gyp), g_x)  # without the weight gradient: the same g_x, bit for bit


@pytest.mark.parametrize("cap,hub", [(256, 0), (256, 16), (128, 0), (1024, 64)])
def test_spmv_edges_per_lane(cap, hub):
    """The SpMV kernel with one, two and four edges per lane (workgroups of cap, cap/2 and cap/4
    lanes) against the oracle: runs of a row inside a lane, across lanes and across wavefronts,
    on R-MAT rows long enough to span a whole part."""
    from paper_1605_02043_amd import Plan

    R = gen.rmat(scale=14, n_edges=1 << 18, seed=7)
    g = spmv_graph(R, R["shuffle"])
    ref = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    A = spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    P = Plan(g["edges"], g["n"], cap, g["w"], kind="spmv", n_x=g["n_x"], class_weight=(1, 4),
             hub_degree=hub).upload("cuda")
    perm = P.perm()
    n_x = g["n_x"]
    xp = torch.from_numpy(np.ascontiguousarray(R["x"][perm[:n_x]])).cuda()
    for ept in (1, 2, 4):
        wg = max(64, -(-cap // ept))
        if -(-cap // wg) != ept:
            continue
        for layout in (0, 1):
            say(f"case spmv ept={ept} cap={cap} hub={hub} wg={wg} layout={layout}")
            P.set_launch(wg)
            P.set_slot_layout(layout)
            y = P.spmv(xp)
            torch.cuda.synchronize()
            out = np.empty(g["n"] - n_x, dtype=np.float32)
            out[perm[n_x:] - n_x] = y.cpu().numpy()
            assert_close(f"spmv14/ept{ept}/{cap}/{hub}/{layout}", out, ref, A)
            assert torch.equal(P.spmv(xp), y)  # launch after launch: the same bits


def test_spmv_adjoint_through_transpose_plan():
    """g_x = A^T g_y as the forward SpMV of a plan of A^T (hub split and weights as the forward's
    plan) against the oracle's adjoint, and close to the same-plan adjoint."""
    from paper_1605_02043_amd import Plan

    R = gen.rmat(scale=14, n_edges=1 << 18, seed=9)
    gy = np.random.default_rng(4).standard_normal(R["n_y"]).astype(np.float32)
    g = spmv_graph(R, R["shuffle"])
    ref, _ = spmv.backward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)
    A, _ = spmv.backward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"], gy)
    RT = {"rows": R["cols"], "cols": R["rows"], "w": R["w"], "n_x": R["n_y"], "n_y": R["n_x"]}
    gt = spmv_graph(RT, R["shuffle"])
    say("case spmv adjoint via the transpose plan")
    PT = Plan(gt["edges"], gt["n"], 256, gt["w"], kind="spmv", n_x=gt["n_x"], class_weight=(1, 4),
              hub_degree=16).upload("cuda")
    perm = PT.perm()
    n_in = gt["n_x"]
    gx = PT.spmv(torch.from_numpy(np.ascontiguousarray(gy[perm[:n_in]])).cuda())
    torch.cuda.synchronize()
    out = np.empty(R["n_x"], dtype=np.float32)
    out[perm[n_in:] - n_in] = gx.cpu().numpy()
    assert_close("spmv14/adjoint-by-transpose", out, ref, A)
    P = Plan(g["edges"], g["n"], 256, g["w"], kind="spmv", n_x=g["n_x"], class_weight=(1, 4),
             hub_degree=16).upload("cuda")
    p2 = P.perm()
    gx2 = P.spmv_adjoint(torch.from_numpy(np.ascontiguousarray(gy[p2[g["n_x"]:] - g["n_x"]])).cuda())
    same = np.empty(R["n_x"], dtype=np.float32)
    same[p2[:g["n_x"]]] = gx2.cpu().numpy()
    assert np.linalg.norm(out.astype(np.float64) - same) <= 1e-5 * np.linalg.norm(same.astype(np.float64))

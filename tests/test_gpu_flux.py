"""GPU parity of the FLUX5 forward and adjoint kernels against the FP64 oracle.

Every call goes through the C ABI (ctypes binding); inputs are packed and
results unpacked on the host with the plan's permutation, so the oracle sees
original vertex ids only.
"""

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


def _plan(G, cap, order="ep"):
    from paper_1605_02043_amd import Plan

    return Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32), order=order).upload("cuda")


def _fwd(P, q, dt=None):
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    out = P.forward(qd, dt)
    torch.cuda.synchronize()
    if dt is None:
        return unpack_rows(out.cpu().numpy(), perm)
    return unpack_rows(out[0].cpu().numpy(), perm), unpack_rows(out[1].cpu().numpy(), perm)


def _bwd(P, q, gr):
    perm = P.perm()
    g = P.backward(torch.from_numpy(pack_rows(q, perm)).cuda(), torch.from_numpy(pack_rows(gr, perm)).cuda())
    torch.cuda.synchronize()
    return unpack_rows(g.cpu().numpy(), perm)


def _geom32(G):
    return G["geom"].astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("order", ["ep", "input"])
def test_forward_grid64(order):
    G = gen.workload("grid64", seed=0)
    say(f"case grid64 order={order} n={G['n']} m={len(G['edges'])}")
    q = gen.flux_state(G["n"], seed=0)
    P = _plan(G, 256, order)
    r, qn = _fwd(P, q, dt=0.01)
    ref, qref = flux.forward(G["n"], G["edges"], _geom32(G), q, dt=0.01)
    A, qA = flux.forward_abs(G["n"], G["edges"], _geom32(G), q, dt=0.01)
    assert_close(f"grid64/{order}/r", r, ref, A)
    assert_close(f"grid64/{order}/q_new", qn, qref, qA)


@pytest.mark.parametrize("order", ["ep", "input"])
@pytest.mark.parametrize("seed", [0, 1])
def test_forward_tet32(order, seed):
    G = gen.workload("tet32", seed=seed)
    say(f"case tet32 order={order} seed={seed}")
    q = gen.flux_state(G["n"], seed=seed)
    P = _plan(G, 256, order)
    r = _fwd(P, q)
    g = _geom32(G)
    assert_close(f"tet32/{order}/r", r, flux.forward(G["n"], G["edges"], g, q), flux.forward_abs(G["n"], G["edges"], g, q))


def test_forward_tet55_full_size_both_orders():
    G = gen.workload("tet55", seed=0)
    say(f"case tet55 n={G['n']} m={len(G['edges'])}")
    q = gen.flux_state(G["n"], seed=0)
    g = _geom32(G)
    ref = flux.forward(G["n"], G["edges"], g, q)
    A = flux.forward_abs(G["n"], G["edges"], g, q)
    for order in ("ep", "input"):
        P = _plan(G, 256, order)
        assert_close(f"tet55/{order}/r", _fwd(P, q), ref, A)


@pytest.mark.parametrize("name,cap", [("grid64", 256), ("tet32", 256), ("tet32", 64), ("tet32", 512)])
def test_backward(name, cap):
    G = gen.workload(name, seed=0)
    say(f"case backward {name} cap={cap}")
    q = gen.flux_state(G["n"], seed=0)
    gr = gen.workloads.grad_seed(G["n"], seed=0)
    P = _plan(G, cap)
    g = _geom32(G)
    ref = flux.backward(G["n"], G["edges"], g, q, gr)
    A = flux.backward_abs(G["n"], G["edges"], g, q, gr)
    assert_close(f"bwd/{name}/{cap}", _bwd(P, q, gr), ref, A)


def test_backward_tet55_full_size():
    G = gen.workload("tet55", seed=0)
    say("case backward tet55")
    q = gen.flux_state(G["n"], seed=0)
    g = _geom32(G)
    r = flux.forward(G["n"], G["edges"], g, q)
    gr = (2.0 * r).astype(np.float32)  # loss = sum r^2, upstream gradient from the oracle
    ref = flux.backward(G["n"], G["edges"], g, q, gr)
    A = flux.backward_abs(G["n"], G["edges"], g, q, gr)
    for order in ("ep", "input"):
        P = _plan(G, 256, order)
        assert_close(f"bwd/tet55/{order}", _bwd(P, q, gr), ref, A)


def test_autograd_matches_finite_differences_on_1k_cells():
    """Loss sum r^2 on the BFS 1k-cell subgraph of the 1M-cell mesh: GPU gradient
    vs FP64 central differences (oracle forward) and vs the oracle adjoint."""
    from paper_1605_02043_amd.autograd import edge_flux

    S = gen.bfs_subgraph(gen.tet_mesh(55, 55, 55, seed=0), 1000)
    say(f"case fd1k n={S['n']} m={len(S['edges'])}")
    q = gen.flux_state(S["n"], seed=3)
    P = _plan(S, 256)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda().requires_grad_(True)
    r = edge_flux(qd, P)
    (r * r).sum().backward()
    g_gpu = unpack_rows(qd.grad.cpu().numpy(), perm)
    g = _geom32(S)
    qq = q.astype(np.float64)
    r64 = flux.forward(S["n"], S["edges"], g, qq)
    ref = flux.backward(S["n"], S["edges"], g, qq, 2.0 * r64)
    A = flux.backward_abs(S["n"], S["edges"], g, qq, 2.0 * np.abs(r64) + 2.0 * flux.forward_abs(S["n"], S["edges"], g, qq))
    assert_close("fd1k/analytic", g_gpu, ref, A)
    rng = np.random.default_rng(0)
    idx = rng.choice(S["n"] * 5, 300, replace=False)
    fd = np.empty(len(idx))
    for t, flat in enumerate(idx):
        i, c = divmod(int(flat), 5)
        h = 1e-6 * max(1.0, abs(qq[i, c]))
        qp, qm = qq.copy(), qq.copy()
        qp[i, c] += h
        qm[i, c] -= h
        fd[t] = (flux.loss(S["n"], S["edges"], g, qp) - flux.loss(S["n"], S["edges"], g, qm)) / (2 * h)
    err = np.linalg.norm(g_gpu.reshape(-1)[idx] - fd) / np.linalg.norm(fd)
    say(f"[fd1k/finite-differences] normwise = {err:.3e}")
    assert err <= 1e-5


def test_bitwise_determinism_and_launch_shapes():
    G = gen.workload("tet32", seed=0)
    q = gen.flux_state(G["n"], seed=0)
    gr = gen.workloads.grad_seed(G["n"], seed=0)
    P = _plan(G, 256)
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    outs = []
    for wg, sw in [(256, 1), (256, 1), (256, 1), (256, 0), (128, 1), (64, 0)]:
        say(f"case determinism wg={wg} swizzle={sw}")
        P.set_launch(wg, sw)
        outs.append((P.forward(qd).cpu(), P.backward(qd, gd).cpu()))
    for r, g in outs[1:]:
        assert torch.equal(r, outs[0][0]) and torch.equal(g, outs[0][1])


# The largest capacity at which tet32's adjoint still fits the 64 KiB of LDS a workgroup
# may ask for (its parts then touch up to 611 vertices; capacity 1024 is refused).
MAX_CAP_TET32 = 896


def test_largest_capacity_that_fits():
    """A maximum-size case: tet32 at the largest capacity whose adjoint fits the LDS budget
    (within 1% of it), forward and adjoint against the oracle, and bitwise the same at one,
    two, four and eight edges per lane."""
    G = gen.workload("tet32", seed=0)
    say(f"case largest capacity tet32 cap={MAX_CAP_TET32}")
    P = _plan(G, MAX_CAP_TET32)
    info = P.info()
    assert 0.99 * 65536 <= info["lds_bwd"] <= 65536 and P.stats["max_part_edges"] == MAX_CAP_TET32
    q = gen.flux_state(G["n"], seed=0)
    gr = gen.workloads.grad_seed(G["n"], seed=0)
    g = _geom32(G)
    assert_close("maxcap/r", _fwd(P, q), flux.forward(G["n"], G["edges"], g, q), flux.forward_abs(G["n"], G["edges"], g, q))
    assert_close("maxcap/g_q", _bwd(P, q, gr), flux.backward(G["n"], G["edges"], g, q, gr),
                 flux.backward_abs(G["n"], G["edges"], g, q, gr))
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    outs = []
    for wg in (1024, 512, 256, 128):
        say(f"  wg={wg}")
        P.set_launch(wg, 1)
        outs.append((P.forward(qd).cpu(), P.backward(qd, gd).cpu()))
    for r, gq in outs[1:]:
        assert torch.equal(r, outs[0][0]) and torch.equal(gq, outs[0][1])


def test_orders_agree():
    G = gen.workload("tet32", seed=2)
    q = gen.flux_state(G["n"], seed=2)
    a = _fwd(_plan(G, 256, "ep"), q)
    b = _fwd(_plan(G, 256, "input"), q)
    A = flux.forward_abs(G["n"], G["edges"], _geom32(G), q)
    assert (np.abs(a - b) <= 2e-5 * (np.abs(b) + A)).all()


# ------------------------------------------------------------------ edge cases

def _small_case(edges, n, cap, dim=3, seed=0, order="ep"):
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
    g = _geom32(G)
    r, qn = _fwd(P, q, dt=-0.5)
    ref, qref = flux.forward(n, edges, g, q, dt=-0.5)
    A, qA = flux.forward_abs(n, edges, g, q, dt=-0.5)
    assert_close("edge/r", r, ref, A)
    assert_close("edge/q_new", qn, qref, qA)
    assert_close("edge/g_q", _bwd(P, q, gr), flux.backward(n, edges, g, q, gr), flux.backward_abs(n, edges, g, q, gr))


def test_edge_empty_graph_zeroes_output():
    say("case empty graph")
    _small_case(np.zeros((0, 2)), 7, 16)


def test_edge_single_edge_and_isolated_vertices():
    say("case single edge + isolated")
    _small_case([[3, 1]], 6, 4)


def test_edge_capacity_one_and_ragged():
    rng = np.random.default_rng(1)
    n, m = 50, 203
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    for cap in (1, 7, 64, 512):
        say(f"case ragged cap={cap}")
        _small_case(np.stack([u, v], 1), n + 5, cap, seed=cap)


def test_edge_2d_geometry_and_hub():
    n = 300
    star = np.stack([np.zeros(n - 1, int), np.arange(1, n)], 1)  # hub in ~all parts
    say("case hub 2D")
    _small_case(star, n, 16, dim=2)
    say("case hub 3D input order")
    _small_case(star, n, 16, order="input")


def test_edge_dense_parts_and_heavy_hub():
    """Parts with more foreign ids and more vertices than a workgroup has lanes (several id,
    row and sum steps per lane; two edges per lane at capacity 512), and a hub with more
    partials than the light reduction path takes (the one-workgroup-per-vertex path)."""
    rng = np.random.default_rng(7)
    n, m = 1200, 5000  # capacity 512: up to 394 foreign ids and 397 vertices in one part
    u = rng.integers(0, n, m)
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    say("case dense parts cap=512")
    _small_case(np.stack([u, v], 1), n, 512, seed=7)
    n = 300
    star = np.stack([np.zeros(n - 1, int), np.arange(1, n)], 1)  # capacity 2: the hub has 149 partials
    say("case heavy hub cap=2")
    _small_case(star, n, 2, dim=2)


def test_permute_rows_roundtrip():
    from paper_1605_02043_amd import permute_rows

    say("case permute")
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal((1000, 5)).astype(np.float32)).cuda()
    perm = torch.from_numpy(rng.permutation(1000).astype(np.int32)).cuda()
    y = permute_rows(x, perm, inverse=False)
    assert torch.equal(y.cpu(), x.cpu()[perm.cpu().long()])
    z = permute_rows(y, perm, inverse=True)
    assert torch.equal(z.cpu(), x.cpu())

"""Seeded random sweep of plans and launch settings against the FP64 oracle.

Each case draws a multigraph (2D or 3D geometry, hubs and isolated vertices
included), a capacity, a task order (EP with or without the hub split, GGP,
input, random, greedy), a workgroup size, a slot layout, the cache-only
variant, the pipelined launch and the single-launch reduction, and checks the
forward (with q_new) and the adjoint against the oracle.  SpMV cases draw a
bipartite power-law graph, class weights, a hub threshold, edges per lane and
a slot layout, and check y = A x and the adjoint.  Combinations the library
refuses (LDS budget, launch limits) are skipped, each refusal checked to be an
EpkError."""

import numpy as np
import pytest

from gen.rmat import spmv_graph
from oracle import flux, spmv
from tests.gpu_util import assert_close, pack_rows, say, unpack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02043_amd import Plan  # noqa: F401  (fails loudly without libepk.so)


def _graph(rng):
    n = int(rng.integers(2, 3000))
    m = int(rng.integers(1, 6000))
    u = rng.integers(0, n, m)
    if rng.random() < 0.5:  # a hub
        u[rng.random(m) < 0.3] = int(rng.integers(0, n))
    v = (u + 1 + rng.integers(0, n - 1, m)) % n
    E = np.stack([u, v], 1).astype(np.int32)
    if rng.random() < 0.5:
        nrm = rng.standard_normal((m, 2))
        geom = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    else:
        nrm = rng.standard_normal((m, 3))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        geom = np.concatenate([nrm, rng.uniform(0.5, 2.0, (m, 1))], 1).astype(np.float32)
    return n + int(rng.integers(0, 4)), E, geom  # a few isolated vertices


def _try(fn):
    from paper_1605_02043_amd._lib import EpkError

    try:
        fn()
        return True
    except EpkError:
        return False


@pytest.mark.parametrize("seed", range(96))
def test_random_flux_plans(seed):
    from paper_1605_02043_amd import Plan

    rng = np.random.default_rng(1000 + seed)
    n, E, geom = _graph(rng)
    cap = int(rng.choice([1, 5, 64, 100, 256, 384]))
    order = str(rng.choice(["ep", "ep", "ggp", "input", "random", "greedy"]))
    hub = int(rng.choice([0, 0, 3, 8])) if order == "ep" else 0
    wgs = [w for w in (64, 128, 192, 256, 512) if cap <= 8 * w]
    wg = int(rng.choice(wgs))
    layout, staging = int(rng.choice([-1, 0, 1])), int(rng.random() < 0.8)
    pipe, fused = int(rng.random() < 0.3), int(rng.random() < 0.3)
    say(f"case random flux seed={seed} n={n} m={len(E)} g={geom.shape[1]} cap={cap} order={order} hub={hub} "
        f"wg={wg} layout={layout} staging={staging} pipe={pipe} fused={fused}")
    P = Plan(E, n, cap, geom, order=order, hub_degree=hub)
    assert P.stats["max_part_edges"] <= cap
    P.set_launch(wg)
    _try(lambda: P.set_slot_layout(layout))
    P.upload("cuda")
    if not staging:
        _try(lambda: P.set_staging(0))
    elif pipe:
        _try(lambda: P.set_pipeline(-1))
    if fused:
        _try(lambda: P.set_fused(1))
    say(f"  info {P.info()}")
    perm = P.perm()
    q = np.random.default_rng(seed).uniform(0.5, 1.5, (n, 5)).astype(np.float32)
    gr = np.random.default_rng(seed + 1).standard_normal((n, 5)).astype(np.float32)
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    dt = -0.01
    r, qn = P.forward(qd, dt)
    g = P.backward(qd, gd)
    torch.cuda.synchronize()
    g64 = geom.astype(np.float64)
    ref = flux.forward(n, E, g64, q)
    A = flux.forward_abs(n, E, g64, q)
    r_h = unpack_rows(r.cpu().numpy(), perm)
    assert_close(f"random{seed}/r", r_h, ref, A)
    assert_close(f"random{seed}/q_new", unpack_rows(qn.cpu().numpy(), perm), q + dt * ref,
                 np.abs(q) + abs(dt) * (np.abs(ref) + A))
    assert_close(f"random{seed}/g_q", unpack_rows(g.cpu().numpy(), perm), flux.backward(n, E, g64, q, gr),
                 flux.backward_abs(n, E, g64, q, gr))


@pytest.mark.parametrize("seed", range(48))
def test_random_spmv_plans(seed):
    from paper_1605_02043_amd import Plan

    rng = np.random.default_rng(2000 + seed)
    n_x, n_y = int(rng.integers(1, 3000)), int(rng.integers(1, 3000))
    m = int(rng.integers(1, 40000))
    py = 1.0 / np.arange(1, n_y + 1) ** rng.uniform(0.5, 1.5)
    R = {"rows": rng.choice(n_y, size=m, p=py / py.sum()).astype(np.int32),
         "cols": rng.integers(0, n_x, m).astype(np.int32), "w": rng.random(m, dtype=np.float32),
         "n_x": n_x, "n_y": n_y}
    g = spmv_graph(R, rng.permutation(m))
    x = rng.standard_normal(n_x).astype(np.float32)
    gy = rng.standard_normal(n_y).astype(np.float32)
    cap = int(rng.choice([1, 33, 64, 256, 1024]))
    order = str(rng.choice(["ep", "ep", "input", "greedy"]))
    cw = (1, int(rng.integers(1, 9))) if order == "ep" and rng.random() < 0.7 else None
    hub = int(rng.choice([0, 4, 16])) if order == "ep" else 0
    wgs = [w for w in (64, 128, 256, 512, 1024) if cap <= 4 * w]
    wg, layout = int(rng.choice(wgs)), int(rng.choice([-1, 0, 1]))
    say(f"case random spmv seed={seed} n_x={n_x} n_y={n_y} m={m} cap={cap} order={order} cw={cw} hub={hub} "
        f"wg={wg} layout={layout}")
    P = Plan(g["edges"], g["n"], cap, g["w"], order=order, kind="spmv", n_x=n_x, class_weight=cw, hub_degree=hub)
    P.set_launch(wg)
    _try(lambda: P.set_slot_layout(layout))
    P.upload("cuda")
    perm = P.perm()
    xp = torch.from_numpy(np.ascontiguousarray(x[perm[:n_x]])).cuda()
    y = P.spmv(xp)
    gyp = torch.from_numpy(np.ascontiguousarray(gy[perm[n_x:] - n_x])).cuda()
    gx = P.spmv_adjoint(gyp)
    torch.cuda.synchronize()
    out = np.empty(n_y, dtype=np.float32)
    out[perm[n_x:] - n_x] = y.cpu().numpy()
    assert_close(f"random-spmv{seed}/y", out, spmv.forward(n_x, n_y, g["edges"], g["w"], x),
                 spmv.forward_abs(n_x, n_y, g["edges"], g["w"], x))
    ox = np.empty(n_x, dtype=np.float32)
    ox[perm[:n_x]] = gx.cpu().numpy()
    assert_close(f"random-spmv{seed}/g_x", ox, spmv.backward(n_x, n_y, g["edges"], g["w"], x, gy)[0],
                 spmv.backward_abs(n_x, n_y, g["edges"], g["w"], x, gy)[0])

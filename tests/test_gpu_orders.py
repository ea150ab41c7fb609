"""GPU parity of the FLUX5 forward and adjoint under every task order the
library builds, and of the whole 256-graph batch at the launch configuration
the autotuner picks.

* tet32 (196,608 cells, 387,072 faces) at capacity 256 under single-pass
  greedy growing (Section 3.2 read as one greedy pass) and under the random
  and greedy vertex-cut placements of Section 3.3's comparison: forward and
  adjoint against the FP64 oracle, and the loads the kernels stage (the
  plan's L) equal the cost the oracle recounts from the same partition.
* batch256, all 256 graphs, forward and adjoint against the oracle, at the
  capacity, workgroup size and launch kind the autotuner returns (the
  configuration the benchmark runs).
"""

import numpy as np
import pytest

import gen
from oracle import cost, flux
from tests.gpu_util import assert_close, pack_rows, say, unpack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02043_amd import Plan  # noqa: F401  (fails loudly without libepk.so)


@pytest.fixture(scope="module")
def tet32():
    G = gen.workload("tet32", seed=1)
    q = gen.flux_state(G["n"], seed=1)
    gr = gen.workloads.grad_seed(G["n"], seed=1)
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    ref = {"r": flux.forward(G["n"], G["edges"], g64, q), "rA": flux.forward_abs(G["n"], G["edges"], g64, q),
           "g": flux.backward(G["n"], G["edges"], g64, q, gr), "gA": flux.backward_abs(G["n"], G["edges"], g64, q, gr)}
    return G, q, gr, ref


@pytest.mark.parametrize("order", ["ggp", "random", "greedy"])
def test_tet32_orders_forward_adjoint(tet32, order):
    from paper_1605_02043_amd import Plan

    G, q, gr, ref = tet32
    say(f"case tet32 order={order} cap=256")
    P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32), order=order).upload("cuda")
    part, _ = P.part_of_edge()
    st = P.stats
    c = cost.partition_cost(G["edges"], G["n"], part, st["n_parts"])
    assert (st["loads"], st["cost"], st["replicated"]) == (c["loads"], c["cost"], c["replicated"])
    assert st["max_part_edges"] <= 256
    say(f"  loads/edge {st['loads'] / len(G['edges']):.3f}")
    perm = P.perm()
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    gd = torch.from_numpy(pack_rows(gr, perm)).cuda()
    r = P.forward(qd)
    g = P.backward(qd, gd)
    torch.cuda.synchronize()
    assert_close(f"tet32/{order}/r", unpack_rows(r.cpu().numpy(), perm), ref["r"], ref["rA"])
    assert_close(f"tet32/{order}/g_q", unpack_rows(g.cpu().numpy(), perm), ref["g"], ref["gA"])


def test_batch256_full_at_tuned_configuration():
    from paper_1605_02043_amd import Plan
    from paper_1605_02043_amd.batch import Batch, autotune

    graphs = gen.batch_graphs(256, seed=0)
    say(f"case batch256 tuned: n={sum(g['n'] for g in graphs)} m={sum(len(g['edges']) for g in graphs)}")
    caps, wgs, directs = autotune(graphs, caps=(64, 128, 256, 512))
    say(f"  tuned: capacity {caps[0]} wg {wgs[0]} direct {directs[0]}")
    plans = [Plan(g["edges"], g["n"], int(c), g["geom"].astype(np.float32)) for g, c in zip(graphs, caps)]
    B = Batch(plans).set_launch(int(wgs[0]), int(directs[0])).upload("cuda")
    info = B.info()
    assert info["wg"] == wgs[0] and info["direct"] == directs[0]
    qs = [gen.flux_state(g["n"], seed=i) for i, g in enumerate(graphs)]
    grs = [gen.workloads.grad_seed(g["n"], seed=i) for i, g in enumerate(graphs)]
    qd = torch.from_numpy(np.concatenate([a[p.perm()] for a, p in zip(qs, plans)])).cuda()
    gd = torch.from_numpy(np.concatenate([a[p.perm()] for a, p in zip(grs, plans)])).cuda()
    r = B.forward(qd).cpu().numpy()
    gq = B.backward(qd, gd).cpu().numpy()
    worst = {"r": 0.0, "g_q": 0.0}
    for i, (g, p) in enumerate(zip(graphs, plans)):
        sl = slice(int(B.offsets[i]), int(B.offsets[i + 1]))
        ri, gi = unpack_rows(r[sl], p.perm()), unpack_rows(gq[sl], p.perm())
        geo = g["geom"].astype(np.float32).astype(np.float64)
        e1 = assert_close(f"batch256/g{i}/r", ri, flux.forward(g["n"], g["edges"], geo, qs[i]),
                          flux.forward_abs(g["n"], g["edges"], geo, qs[i]))
        e2 = assert_close(f"batch256/g{i}/g_q", gi, flux.backward(g["n"], g["edges"], geo, qs[i], grs[i]),
                          flux.backward_abs(g["n"], g["edges"], geo, qs[i], grs[i]))
        worst["r"] = max(worst["r"], e1["elementwise"])
        worst["g_q"] = max(worst["g_q"], e2["elementwise"])
    say(f"  worst elementwise over the 256 graphs: {worst}")

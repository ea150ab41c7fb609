"""GPU check of epk_forward_scratch, the forward for callers that cannot allocate.

It runs the same kernels as epk_forward with the replicated-vertex partials in
the library's fixed per-device array instead of a caller workspace.  Two calls
in a row, the second on a smaller graph (the array keeps the first call's
contents), each compared with epk_forward on the same inputs through the C ABI:
r and q_new bit for bit, and r against the FP64 oracle at the 1e-5 bar.
"""

import ctypes as C

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


def _both(G, cap, seed, dt):
    from paper_1605_02043_amd import Plan
    from paper_1605_02043_amd._lib import check, lib

    P = Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32)).upload("cuda")
    img, ws = P.device_bytes()
    say(f"  plan: n={G['n']} m={len(G['edges'])} parts={P.stats['n_parts']} workspace={ws} B")
    perm = P.perm()
    q = gen.flux_state(G["n"], seed=seed)
    qd = torch.from_numpy(pack_rows(q, perm)).cuda()
    r_ref, qn_ref = torch.empty_like(qd), torch.empty_like(qd)
    r_s, qn_s = torch.full_like(qd, float("nan")), torch.full_like(qd, float("nan"))
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    check(lib.epk_forward(P._h, ptr(qd), ptr(r_ref), C.c_float(dt), ptr(qn_ref), ptr(P.workspace), s))
    check(lib.epk_forward_scratch(P._h, ptr(qd), ptr(r_s), C.c_float(dt), ptr(qn_s), s))
    torch.cuda.synchronize()
    assert torch.equal(r_s, r_ref), "r differs from epk_forward"
    assert torch.equal(qn_s, qn_ref), "q_new differs from epk_forward"
    g64 = G["geom"].astype(np.float32).astype(np.float64)
    r = unpack_rows(r_s.cpu().numpy(), perm)
    assert_close("scratch/r", r, flux.forward(G["n"], G["edges"], g64, q), flux.forward_abs(G["n"], G["edges"], g64, q))
    return ws


def test_forward_scratch_two_calls_second_smaller():
    big = gen.tet_mesh(24, 24, 24, seed=4)
    small = gen.grid2d(40, 30, seed=5)
    say("case scratch call 1: tet mesh 24^3, capacity 256")
    ws1 = _both(big, 256, 1, 0.01)
    say("case scratch call 2: 2D grid 40x30, capacity 128")
    ws2 = _both(small, 128, 2, -0.02)
    assert ws2 < ws1

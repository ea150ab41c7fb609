"""The benchmarking call epk_run_stage_timed: each stage's kernel timed by its own dispatch
timestamps gives the results of epk_run_stage bit for bit, a positive duration for a stage
that launches a kernel and zero for one that launches none (stage 1 under the single-launch
reduction), on FLUX5 and SpMV plans."""

import ctypes as C

import numpy as np
import pytest

import gen
from gen.rmat import spmv_graph
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02043_amd import Plan  # noqa: F401  (fails loudly without libepk.so)


def _timed(P, op, stage, a, b, out):
    from paper_1605_02043_amd._lib import check, lib
    from paper_1605_02043_amd.plan import _dptr

    ms = C.c_float(-1.0)
    h = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib.epk_run_stage_timed(P._h, op, stage, _dptr(a), _dptr(b), _dptr(out), 0.0, None, _dptr(P.workspace), h,
                                  C.byref(ms)))
    return ms.value


@pytest.mark.parametrize("fused", [0, 1])
def test_timed_stages_flux(fused):
    from paper_1605_02043_amd import Plan

    G = gen.workload("tet32", seed=0)
    say(f"case timed flux tet32 fused={fused}")
    P = Plan(G["edges"], G["n"], 256, G["geom"].astype(np.float32)).upload("cuda")
    P.set_fused(fused)
    q = torch.from_numpy(gen.flux_state(G["n"], seed=3)[P.perm()]).cuda()
    r0 = P.forward(q)
    g0 = P.backward(q, r0)
    torch.cuda.synchronize()
    r = torch.full_like(q, float("nan"))
    g = torch.full_like(q, float("nan"))
    t = [_timed(P, 0, 0, q, None, r), _timed(P, 0, 1, q, None, r), _timed(P, 1, 0, q, r, g), _timed(P, 1, 1, q, r, g)]
    torch.cuda.synchronize()
    assert torch.equal(r, r0) and torch.equal(g, g0)
    assert 0 < t[0] < 50 and 0 < t[2] < 50, t
    if fused:
        assert t[1] == 0 and t[3] == 0
    else:
        assert 0 < t[1] < 50 and 0 < t[3] < 50, t


def test_timed_stages_spmv():
    from paper_1605_02043_amd import Plan

    R = gen.rmat(14, 1 << 17, seed=2)
    g = spmv_graph(R, R["shuffle"])
    say("case timed spmv rmat14")
    P = Plan(g["edges"], g["n"], 256, g["w"], kind="spmv", n_x=g["n_x"]).upload("cuda")
    x = torch.from_numpy(np.ascontiguousarray(R["x"][P.perm()[:R["n_x"]]])).cuda()
    y0 = P.spmv(x)
    torch.cuda.synchronize()
    y = torch.full_like(y0, float("nan"))
    t = [_timed(P, 2, 0, x, None, y), _timed(P, 2, 1, x, None, y)]
    assert torch.equal(y, y0)
    assert all(0 < v < 50 for v in t), t

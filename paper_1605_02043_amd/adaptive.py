"""Adaptive overhead control (the paper's EP-adapt, Sections 4.2 and 5).

The application starts at once in its default task order; the partitioned
plan is built on a background CPU thread inside libepk (epk_adaptive_*).  When
it is ready, one step is timed on each plan and the faster one is kept; the
state moves to the new plan's packed order with one device permutation.
"""

from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib
from ._lib import EpkError, check, lib
from .plan import Plan, _full_device, make_graph

STATES = {0: "running", 1: "ready", 2: "skipped", 3: "failed"}


class AdaptivePartition:
    """Background EP partition of a graph: poll(), take() -> Plan or None."""

    def __init__(self, edges, n: int, cap: int, geom, kind: str = "flux5", n_x: int = 0, min_saving: float = 0.1):
        self.n, self.m, self.cap, self.kind, self.n_x = int(n), int(len(edges)), int(cap), kind, int(n_x)
        gs, keep = make_graph(edges, n, geom, n_x)
        h = C.c_void_p()
        check(lib.epk_adaptive_start(C.byref(gs), int(cap), _lib.KIND[kind], float(min_saving), C.byref(h)))
        del keep  # the library copied the arrays
        self._h = h

    def poll(self) -> dict:
        st = C.c_int32()
        sav, sec = C.c_double(), C.c_double()
        check(lib.epk_adaptive_poll(self._h, C.byref(st), C.byref(sav), C.byref(sec)))
        return {"state": STATES[st.value], "saving_bound": sav.value, "seconds": sec.value}

    def take(self, wait: bool = False):
        """The partitioned plan once ready (None while running or if skipped)."""
        ph = C.c_void_p()
        s = lib.epk_adaptive_take(self._h, int(bool(wait)), C.byref(ph))
        if s == _lib.EPK_OK:
            return Plan._adopt(ph, self.n, self.m, self.cap, self.kind, self.n_x)
        msg = lib.epk_last_error()
        if s == _lib.EPK_ESTATE and self.poll()["state"] in ("running", "skipped"):
            return None
        raise EpkError(s, msg.decode() if msg else "")

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.epk_adaptive_destroy(h)
            self._h = None

    __del__ = close


class AdaptiveFlux:
    """FLUX5 steps that start in the default order and switch to the partitioned order
    when its plan is ready and times faster on the device.

    ``q`` handed to forward/backward is in the current plan's packed order; ``pack`` /
    ``unpack`` convert from / to original vertex order; ``maybe_switch(q)`` returns q in
    the (possibly new) current order.
    """

    def __init__(self, edges, n: int, cap: int, geom, device="cuda", min_saving: float = 0.1):
        import torch

        self.torch = torch
        self.device = _full_device(torch, device)
        self.plan = Plan(edges, n, cap, geom, order="input").upload(self.device)
        self.order = "input"
        self.bg = AdaptivePartition(edges, n, cap, geom, min_saving=min_saving)
        self.decision = None  # set once both orders have been timed (or the partition was skipped)
        self.timings = {}

    def pack(self, q_orig: np.ndarray):
        return self.torch.from_numpy(np.ascontiguousarray(q_orig[self.plan.perm()], dtype=np.float32)).to(self.device)

    def unpack(self, q_packed) -> np.ndarray:
        out = np.empty(q_packed.shape, dtype=np.float32)
        out[self.plan.perm()] = q_packed.cpu().numpy()
        return out

    def forward(self, q, dt=None):
        return self.plan.forward(q, dt)

    def backward(self, q, g_r):
        return self.plan.backward(q, g_r)

    def _time(self, plan, q, reps=3):
        torch = self.torch
        plan.forward(q)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.forward(q)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def maybe_switch(self, q):
        """Poll the background partition; on its first readiness time both orders and keep the faster."""
        if self.decision is not None:
            return q
        st = self.bg.poll()["state"]
        if st == "running":
            return q
        ep = self.bg.take(wait=False) if st == "ready" else None
        if ep is None:
            self.decision = "input (partition " + st + ")"
            return q
        ep.upload(self.device)
        # the state in the partitioned plan's packed order: row i holds original vertex ep.perm[i]
        inv = np.empty(self.plan.n, dtype=np.int64)
        inv[self.plan.perm()] = np.arange(self.plan.n)
        idx = self.torch.from_numpy(inv[ep.perm()].astype(np.int32)).to(self.device)
        from .plan import permute_rows

        q_ep = permute_rows(q, idx, inverse=False)
        self.timings = {"input_ms": self._time(self.plan, q), "ep_ms": self._time(ep, q_ep)}
        if self.timings["ep_ms"] < self.timings["input_ms"]:
            self.plan, self.order, q = ep, "ep", q_ep
        self.decision = self.order
        return q

    def close(self):
        self.bg.close()

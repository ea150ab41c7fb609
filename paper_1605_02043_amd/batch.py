"""Many FLUX5 graphs in one launch per pass, and capacity and launch-shape autotuning."""

from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import Graph, check, i32p, i64p, lib
from .plan import Plan, _dptr, _full_device, _stream_handle, check_tensor, make_graph


class Batch:
    """Merged device image of several FLUX5 plans (4 geometry floats each).

    States of graph g occupy rows [offsets[g], offsets[g+1]) of one [sum n][5]
    tensor, in graph g's packed order.
    """

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = C.c_void_p()
        check(lib.epk_batch_create(len(self.plans), arr, C.byref(h)))
        self._h = h
        off = np.zeros(len(self.plans) + 1, dtype=np.int64)
        check(lib.epk_batch_vertex_offsets(self._h, i64p(off)))
        self.offsets = off
        self.n = int(off[-1])
        self.image = self.workspace = self.device = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.epk_batch_destroy(h)
            self._h = None

    def device_bytes(self):
        a, b = C.c_size_t(), C.c_size_t()
        check(lib.epk_batch_device_bytes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def info(self) -> dict:
        a = np.zeros(10, dtype=np.int64)
        check(lib.epk_batch_info(self._h, i64p(a), 10))
        return dict(zip(["items", "grid", "lds_fwd", "bytes_fwd", "bytes_bwd", "wg", "m", "grid_bwd", "direct",
                         "direct_ok"], a.tolist()))

    def set_launch(self, wg: int = 0, direct: int = -1):
        """Launch shape: workgroup size (64..256, multiple of 64; 0 keeps it) and launch kind
        (direct=1: one workgroup per (graph, part) item; 0: pipelined persistent; -1 keeps it)."""
        check(lib.epk_batch_set_launch(self._h, int(wg), int(direct)))
        return self

    def upload(self, device="cuda"):
        import torch

        dev = _full_device(torch, device)
        img, ws = self.device_bytes()
        self.image = torch.empty(img, dtype=torch.uint8, device=dev)
        self.workspace = torch.empty(max(ws, 4), dtype=torch.uint8, device=dev)
        self.device = dev
        check(lib.epk_batch_upload(self._h, _dptr(self.image), _stream_handle(torch, dev)))
        return self

    def _check_state(self, t, name):
        if self.device is None:
            raise ValueError("batch is not uploaded")
        check_tensor(t, self.device, self.n, 5, name)

    def forward(self, q, out=None):
        """r for the concatenated packed states q[sum n][5] of all graphs."""
        import torch

        self._check_state(q, "q")
        if out is not None:
            self._check_state(out, "out")
        r = out if out is not None else torch.empty_like(q)
        check(lib.epk_batch_forward(self._h, _dptr(q), _dptr(r), _dptr(self.workspace),
                                    _stream_handle(torch, self.device)))
        return r

    def backward(self, q, g_r, out=None):
        """g_q = (dr/dq)^T g_r for the concatenated packed q, g_r [sum n][5]."""
        import torch

        self._check_state(q, "q")
        self._check_state(g_r, "g_r")
        if out is not None:
            self._check_state(out, "out")
        g_q = out if out is not None else torch.empty_like(q)
        check(lib.epk_batch_backward(self._h, _dptr(q), _dptr(g_r), _dptr(g_q), _dptr(self.workspace),
                                     _stream_handle(torch, self.device)))
        return g_q


def autotune(graphs, caps=(64, 128, 256, 512), cache_path=None, device="cuda", scratch_bytes=None):
    """Pick the batch's capacity and launch shape by timing the batched forward + adjoint launch
    at each candidate.

    graphs: list of dicts with 'edges', 'n', 'geom'.  Returns (caps, wgs, directs), each
    [n_graphs]: one capacity, one workgroup size and one launch kind (1: one workgroup per item,
    0: pipelined persistent) for all graphs (the batched launch sizes every workgroup for its
    largest parts); apply the shape with Batch.set_launch(wgs[0], directs[0]).
    """
    import torch

    keep = []
    arr = (Graph * len(graphs))()
    need = 0
    for i, g in enumerate(graphs):
        gs, k = make_graph(g["edges"], g["n"], g["geom"])
        arr[i] = gs
        keep.append(k)
        need += len(g["edges"]) * 160 + g["n"] * 80  # a whole batch's image, workspace and states
    scratch = torch.empty(scratch_bytes or need + (64 << 20), dtype=torch.uint8, device=device)
    c = np.asarray(caps, dtype=np.int32)
    out_cap = np.zeros(len(graphs), dtype=np.int32)
    out_wg = np.zeros(len(graphs), dtype=np.int32)
    out_direct = np.zeros(len(graphs), dtype=np.int32)
    check(lib.epk_autotune(arr, len(graphs), i32p(c), len(c), cache_path.encode() if cache_path else None,
                           _dptr(scratch), scratch.numel(), _stream_handle(torch, _full_device(torch, device)),
                           i32p(out_cap), i32p(out_wg), i32p(out_direct)))
    del keep
    return out_cap, out_wg, out_direct


__all__ = ["Batch", "autotune", "Plan"]

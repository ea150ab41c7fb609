"""Plans (partition + packing + device image) and their device calls.

PyTorch supplies device memory and the stream; every computation runs in
libepk's kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import Graph, Stats, check, i32p, i64p, lib


def make_graph(edges: np.ndarray, n: int, geom: np.ndarray | None = None, n_x: int = 0):
    """A Graph struct plus the arrays it points to (kept alive by the caller)."""
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    g = None
    ncomp = 0
    if geom is not None:
        geom = np.ascontiguousarray(geom, dtype=np.float32)
        if geom.ndim == 1:
            geom = geom.reshape(-1, 1)
        elif len(edges):
            geom = geom.reshape(len(edges), -1)
        ncomp = geom.shape[1]
    gs = Graph(n_vertices=int(n), n_x=int(n_x), n_edges=len(edges), edge_uv=i32p(edges),
               edge_geom=geom.ctypes.data_as(C.POINTER(C.c_float)) if geom is not None else None, geom_ncomp=ncomp)
    return gs, (edges, geom, g)


def _class_weight(class_weight):
    if class_weight is None:
        return None
    w = np.ascontiguousarray(class_weight, dtype=np.int32)
    if w.shape != (2,):
        raise ValueError("class_weight must be two integers (x class, y class)")
    return w


def _hub_degree(order, hub_degree):
    h = int(hub_degree)
    if h < 0:
        raise ValueError("hub_degree must be >= 0")
    if h and order != "ep":
        raise ValueError("the hub split applies to the EP order only")
    return h


def partition(edges: np.ndarray, n: int, cap: int, order: str = "ep", class_weight=None, n_x: int = 0,
              hub_degree: int = 0):
    """Edge partition (host): returns (part[m], task_order[m], stats dict).  class_weight
    (EP order): per-class vertex weights {x, y}, x being the vertices below n_x.  hub_degree > 0
    (EP order): the hub split first (the edges of class-y vertices of higher degree in runs of
    cap, in vertex order)."""
    gs, keep = make_graph(edges, n, None, n_x)
    m = gs.n_edges
    part = np.empty(m, dtype=np.int32)
    task = np.empty(m, dtype=np.int32)
    st = Stats()
    w = _class_weight(class_weight)
    h = _hub_degree(order, hub_degree)
    if h:
        check(lib.epk_partition_hub(C.byref(gs), int(cap), i32p(w), h, i32p(part), i32p(task), C.byref(st)))
    else:
        check(lib.epk_partition_weighted(C.byref(gs), int(cap), _lib.ORDER[order], i32p(w), i32p(part), i32p(task),
                                         C.byref(st)))
    del keep
    return part, task, st.as_dict()


def check_tensor(t, device, rows, cols, name):
    """A device buffer handed to the kernels: a contiguous float32 tensor on `device` of
    shape (rows, cols), or of rows elements when cols == 1."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor")
    if t.device != device or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on {device}")
    if cols == 1:
        if t.numel() != rows:
            raise ValueError(f"{name} must have {rows} elements")
    elif tuple(t.shape) != (rows, cols):
        raise ValueError(f"{name} must have shape ({rows}, {cols})")


def _full_device(torch, device):
    """torch.device with an explicit index ('cuda' -> 'cuda:<current>')."""
    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    return dev


def _stream_handle(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """A partitioned, packed graph ready for the device kernels.

    kind 'flux5': edges [m,2] with geometry [m,2] (nx, ny) or [m,4] (nx, ny, nz, area).
    kind 'spmv' : edges (j, n_x + i) with geometry [m] = the weights.
    States handed to the device calls are in PACKED vertex order.
    """

    def __init__(self, edges, n: int, cap: int, geom, order: str = "ep", kind: str = "flux5", n_x: int = 0,
                 class_weight=None, hub_degree: int = 0):
        self.kind = kind
        self.n = int(n)
        self.n_x = int(n_x)
        self.m = int(len(edges))
        self.cap = int(cap)
        self._h = None
        gs, keep = make_graph(edges, n, geom, n_x)
        h = C.c_void_p()
        w = _class_weight(class_weight)
        hd = _hub_degree(order, hub_degree)
        if hd:
            check(lib.epk_plan_create_hub(C.byref(gs), int(cap), _lib.KIND[kind], i32p(w), hd, C.byref(h)))
        else:
            check(lib.epk_plan_create_weighted(C.byref(gs), int(cap), _lib.ORDER[order], _lib.KIND[kind], i32p(w),
                                               C.byref(h)))
        del keep
        self._h = h
        self.image = None
        self.workspace = None
        self.device = None

    @classmethod
    def from_partition(cls, edges, n: int, cap: int, geom, part, task=None, n_parts: int | None = None,
                       kind: str = "flux5", n_x: int = 0):
        """Plan from a caller's edge partition (part[m] in [0, n_parts); task: the edges part by
        part, parts ascending, or None for ascending edge id inside a part).  A part holding more
        than cap edges is refused (EpkError, status EPK_ERANGE)."""
        self = cls.__new__(cls)
        self.kind, self.n, self.n_x, self.m, self.cap = kind, int(n), int(n_x), int(len(edges)), int(cap)
        part = np.ascontiguousarray(part, dtype=np.int32)
        if part.shape != (self.m,):
            raise ValueError(f"part must have {self.m} entries")
        if task is not None:
            task = np.ascontiguousarray(task, dtype=np.int32)
            if task.shape != (self.m,):
                raise ValueError(f"task must have {self.m} entries")
        k = int(n_parts) if n_parts is not None else (int(part.max()) + 1 if self.m else 0)
        gs, keep = make_graph(edges, n, geom, n_x)
        h = C.c_void_p()
        self._h = None
        check(lib.epk_plan_create_partitioned(C.byref(gs), int(cap), k, i32p(part), i32p(task), _lib.KIND[kind],
                                              C.byref(h)))
        del keep
        self._h = h
        self.image = self.workspace = self.device = None
        return self

    @classmethod
    def _adopt(cls, handle, n: int, m: int, cap: int, kind: str = "flux5", n_x: int = 0):
        """Wrap a plan built elsewhere in the library (the adaptive handle); takes ownership."""
        self = cls.__new__(cls)
        self.kind, self.n, self.n_x, self.m, self.cap = kind, int(n), int(n_x), int(m), int(cap)
        self._h = handle
        self.image = self.workspace = self.device = None
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.epk_plan_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- host queries
    @property
    def stats(self) -> dict:
        st = Stats()
        check(lib.epk_plan_stats(self._h, C.byref(st)))
        return st.as_dict()

    def info(self) -> dict:
        a = np.zeros(17, dtype=np.int64)
        check(lib.epk_plan_info(self._h, i64p(a), 17))
        keys = ["n_parts", "lds_fwd", "lds_bwd", "wg", "ncls", "bytes_fwd", "bytes_bwd", "bytes_fwd_kernel",
                "bytes_bwd_kernel", "max_nf", "pipe", "grid_pipe_fwd", "grid_pipe_bwd", "lds_pipe_bwd",
                "vertex_major", "staging", "fused"]
        return dict(zip(keys, a.tolist()))

    def perm(self) -> np.ndarray:
        p = np.empty(self.n, dtype=np.int32)
        check(lib.epk_plan_vertex_perm(self._h, i32p(p)))
        return p

    def part_of_edge(self):
        part = np.empty(self.m, dtype=np.int32)
        task = np.empty(self.m, dtype=np.int32)
        check(lib.epk_plan_part_of_edge(self._h, i32p(part), i32p(task)))
        return part, task

    def layout(self) -> dict:
        st = self.stats
        k = st["n_parts"]
        ncls = 2 if self.kind == "spmv" else 1
        ob = np.empty(k * ncls, dtype=np.int32)
        oc = np.empty(k * ncls, dtype=np.int32)
        fo = np.empty(k * ncls + 1, dtype=np.int64)
        fi = np.empty(st["cost"], dtype=np.int32)
        check(lib.epk_plan_layout(self._h, i32p(ob), i32p(oc), i64p(fo), i32p(fi)))
        return {"own_begin": ob.reshape(k, ncls), "own_count": oc.reshape(k, ncls), "foreign_offset": fo,
                "foreign_ids": fi}

    def device_bytes(self):
        a, b = C.c_size_t(), C.c_size_t()
        check(lib.epk_plan_device_bytes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_launch(self, wg: int = 0, xcd_swizzle: int = -1):
        """Workgroup size and XCD-aware part mapping; switches the pipelined launch off."""
        check(lib.epk_plan_set_launch(self._h, int(wg), int(xcd_swizzle)))

    def set_staging(self, staged: int = 1):
        """FLUX5: stage states in LDS (1) or read them through the caches only (0)."""
        check(lib.epk_plan_set_staging(self._h, int(staged)))

    def set_slot_layout(self, layout: int = -1):
        """Workspace layout of the replicated partials: 0 part-major, 1 vertex-major, -1 automatic."""
        check(lib.epk_plan_set_slot_layout(self._h, int(layout)))

    def set_fused(self, on: int = 1):
        """FLUX5: sum replicated vertices inside the part kernel (1) or in a second launch (0)."""
        check(lib.epk_plan_set_fused(self._h, int(on)))

    def set_pipeline(self, blocks_per_cu: int = -1):
        """FLUX5: pipelined persistent launch with blocks_per_cu workgroups per CU (-1: as many as
        fit, 0: one workgroup per part).  Needs a current device; call after set_launch."""
        check(lib.epk_plan_set_pipeline(self._h, int(blocks_per_cu)))

    # ---------------------------------------------------------------- device
    def upload(self, device="cuda"):
        import torch

        dev = _full_device(torch, device)
        img, ws = self.device_bytes()
        self.image = torch.empty(img, dtype=torch.uint8, device=dev)
        self.workspace = torch.empty(max(ws, 4), dtype=torch.uint8, device=dev)
        self.device = dev
        check(lib.epk_plan_upload(self._h, _dptr(self.image), _stream_handle(torch, dev)))
        return self

    def _check_state(self, t, rows, cols, name):
        if self.device is None:
            raise ValueError("plan is not uploaded")
        check_tensor(t, self.device, rows, cols, name)

    def forward(self, q, dt: float | None = None, out=None):
        """r (and q_new = q + dt r if dt is given) for packed states q[n][5]."""
        import torch

        self._check_state(q, self.n, 5, "q")
        if out is not None:
            self._check_state(out, self.n, 5, "out")
        r = out if out is not None else torch.empty_like(q)
        qn = torch.empty_like(q) if dt is not None else None
        check(lib.epk_forward(self._h, _dptr(q), _dptr(r), float(dt or 0.0), _dptr(qn), _dptr(self.workspace),
                              _stream_handle(torch, self.device)))
        return (r, qn) if dt is not None else r

    def backward(self, q, g_r, out=None):
        """g_q = (dr/dq)^T g_r for packed q, g_r [n][5]."""
        import torch

        self._check_state(q, self.n, 5, "q")
        self._check_state(g_r, self.n, 5, "g_r")
        if out is not None:
            self._check_state(out, self.n, 5, "out")
        g_q = out if out is not None else torch.empty_like(q)
        check(lib.epk_backward(self._h, _dptr(q), _dptr(g_r), _dptr(g_q), _dptr(self.workspace),
                               _stream_handle(torch, self.device)))
        return g_q

    def spmv(self, x, out=None):
        """y = A x with x in packed x order [n_x] and y in packed y order [n - n_x]."""
        import torch

        self._check_state(x, self.n_x, 1, "x")
        if out is not None:
            self._check_state(out, self.n - self.n_x, 1, "out")
        y = out if out is not None else torch.empty(self.n - self.n_x, dtype=torch.float32, device=self.device)
        check(lib.epk_spmv(self._h, _dptr(x), _dptr(y), _dptr(self.workspace), _stream_handle(torch, self.device)))
        return y

    def spmv_adjoint(self, g_y, x=None, weights_grad: bool = False):
        """g_x = A^T g_y (packed x order) and, with weights_grad, g_w[e] = g_y[i] x[j] in
        original edge order (x, packed, is then required)."""
        import torch

        self._check_state(g_y, self.n - self.n_x, 1, "g_y")
        if weights_grad:
            self._check_state(x, self.n_x, 1, "x")
        g_x = torch.empty(self.n_x, dtype=torch.float32, device=self.device)
        g_w = torch.empty(self.m, dtype=torch.float32, device=self.device) if weights_grad else None
        check(lib.epk_spmv_adjoint(self._h, _dptr(x if weights_grad else None), _dptr(g_y), _dptr(g_x), _dptr(g_w),
                                   _dptr(self.workspace), _stream_handle(torch, self.device)))
        return (g_x, g_w) if weights_grad else g_x

    # ---------------------------------------------------------------- packing
    def pack(self, state_orig, perm_dev=None):
        """Rows of state_orig (original vertex order) -> packed order."""
        return permute_rows(state_orig, self._perm_dev(perm_dev), inverse=False)

    def unpack(self, state_packed, perm_dev=None):
        return permute_rows(state_packed, self._perm_dev(perm_dev), inverse=True)

    def _perm_dev(self, perm_dev):
        import torch

        if perm_dev is None:
            if getattr(self, "_perm_t", None) is None:
                self._perm_t = torch.from_numpy(self.perm()).to(self.device)
            perm_dev = self._perm_t
        return perm_dev


def permute_rows(src, idx, inverse: bool):
    """dst[i] = src[idx[i]] (or dst[idx[i]] = src[i] if inverse), by the library kernel."""
    import torch

    rows = idx.numel()
    ncomp = src.numel() // max(rows, 1) if rows else 1
    dst = torch.empty_like(src)
    check(lib.epk_permute_rows(_dptr(src), _dptr(dst), _dptr(idx), rows, ncomp, int(inverse),
                               _stream_handle(torch, src.device)))
    return dst

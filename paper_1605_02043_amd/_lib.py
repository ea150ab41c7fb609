"""ctypes binding of libepk (include/epk.h).  Argument marshalling only."""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepk.so")

EPK_OK, EPK_EINVAL, EPK_ERANGE, EPK_EHIP, EPK_ESTATE, EPK_ENOMEM, EPK_ECANCELED = 0, -1, -2, -3, -4, -5, -6
ORDER = {"ep": 0, "input": 1, "ggp": 2, "random": 3, "greedy": 4}
KIND = {"flux5": 0, "spmv": 1}


class EpkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"epk status {status}: {msg}")
        self.status = status


class Graph(C.Structure):
    _fields_ = [
        ("n_vertices", C.c_int32),
        ("n_x", C.c_int32),
        ("n_edges", C.c_int64),
        ("edge_uv", C.POINTER(C.c_int32)),
        ("edge_geom", C.POINTER(C.c_float)),
        ("geom_ncomp", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("n_parts", "loads", "cost", "replicated", "slots", "aux_cut", "n_active",
                                         "max_part_edges", "max_part_vertices")] + \
               [(f, C.c_double) for f in ("balance", "partition_seconds", "plan_seconds")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_FP = C.c_void_p  # device float*
_SZP = C.POINTER(C.c_size_t)

_SIGS = {
    "epk_partition": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, _I32P, _I32P, C.POINTER(Stats)]),
    "epk_partition_weighted": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, _I32P, _I32P, _I32P,
                                         C.POINTER(Stats)]),
    "epk_partition_hub": (C.c_int, [C.POINTER(Graph), C.c_int32, _I32P, C.c_int32, _I32P, _I32P, C.POINTER(Stats)]),
    "epk_plan_create": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "epk_plan_create_hub": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, _I32P, C.c_int32, C.POINTER(_P)]),
    "epk_plan_create_weighted": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, C.c_int32, _I32P, C.POINTER(_P)]),
    "epk_plan_create_partitioned": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int64, _I32P, _I32P, C.c_int32,
                                              C.POINTER(_P)]),
    "epk_plan_device_bytes": (C.c_int, [_P, _SZP, _SZP]),
    "epk_plan_upload": (C.c_int, [_P, _P, _P]),
    "epk_plan_vertex_perm": (C.c_int, [_P, _I32P]),
    "epk_plan_part_of_edge": (C.c_int, [_P, _I32P, _I32P]),
    "epk_plan_layout": (C.c_int, [_P, _I32P, _I32P, _I64P, _I32P]),
    "epk_plan_stats": (C.c_int, [_P, C.POINTER(Stats)]),
    "epk_plan_info": (C.c_int, [_P, _I64P, C.c_int32]),
    "epk_plan_set_launch": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "epk_plan_set_pipeline": (C.c_int, [_P, C.c_int32]),
    "epk_plan_set_slot_layout": (C.c_int, [_P, C.c_int32]),
    "epk_plan_set_staging": (C.c_int, [_P, C.c_int32]),
    "epk_plan_set_fused": (C.c_int, [_P, C.c_int32]),
    "epk_plan_destroy": (None, [_P]),
    "epk_forward": (C.c_int, [_P, _FP, _FP, C.c_float, _FP, _P, _P]),
    "epk_forward_scratch": (C.c_int, [_P, _FP, _FP, C.c_float, _FP, _P]),
    "epk_backward": (C.c_int, [_P, _FP, _FP, _FP, _P, _P]),
    "epk_spmv": (C.c_int, [_P, _FP, _FP, _P, _P]),
    "epk_spmv_adjoint": (C.c_int, [_P, _FP, _FP, _FP, _FP, _P, _P]),
    "epk_run_stage": (C.c_int, [_P, C.c_int32, C.c_int32, _FP, _FP, _FP, C.c_float, _FP, _P, _P]),
    "epk_run_stage_timed": (C.c_int, [_P, C.c_int32, C.c_int32, _FP, _FP, _FP, C.c_float, _FP, _P, _P,
                                      C.POINTER(C.c_float)]),
    "epk_permute_rows": (C.c_int, [_FP, _FP, _P, C.c_int64, C.c_int32, C.c_int32, _P]),
    "epk_batch_create": (C.c_int, [C.c_int32, C.POINTER(_P), C.POINTER(_P)]),
    "epk_batch_device_bytes": (C.c_int, [_P, _SZP, _SZP]),
    "epk_batch_upload": (C.c_int, [_P, _P, _P]),
    "epk_batch_set_launch": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "epk_batch_vertex_offsets": (C.c_int, [_P, _I64P]),
    "epk_batch_info": (C.c_int, [_P, _I64P, C.c_int32]),
    "epk_batch_forward": (C.c_int, [_P, _FP, _FP, _P, _P]),
    "epk_batch_backward": (C.c_int, [_P, _FP, _FP, _FP, _P, _P]),
    "epk_batch_destroy": (None, [_P]),
    "epk_autotune": (C.c_int, [C.POINTER(Graph), C.c_int32, _I32P, C.c_int32, C.c_char_p, _P, C.c_size_t, _P,
                               _I32P, _I32P, _I32P]),
    "epk_adaptive_start": (C.c_int, [C.POINTER(Graph), C.c_int32, C.c_int32, C.c_double, C.POINTER(_P)]),
    "epk_adaptive_poll": (C.c_int, [_P, _I32P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "epk_adaptive_take": (C.c_int, [_P, C.c_int32, C.POINTER(_P)]),
    "epk_adaptive_destroy": (None, [_P]),
    "epk_last_error": (C.c_char_p, []),
    "epk_version": (C.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1605_02043_amd/build.py`")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 and owns
    # the device memory and streams handed to libepk, so torch's copy must be the
    # one loaded before libepk.so binds its libamdhip64.so.7 dependency.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int) -> None:
    if status != EPK_OK:
        msg = lib.epk_last_error()
        raise EpkError(status, msg.decode() if msg else "")


def i32p(a):
    return a.ctypes.data_as(_I32P) if a is not None else None


def i64p(a):
    return a.ctypes.data_as(_I64P) if a is not None else None


def fptr_host(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None

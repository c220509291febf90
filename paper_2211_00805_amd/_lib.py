"""ctypes loader for libgeosink.so: signatures of every C entry point.

Importing this module loads the in-tree shared library and raises ImportError
when it has not been built; nothing in this package falls back to another
implementation.
"""
from __future__ import annotations

import ctypes as C
import os

# torch ships its own HIP runtime (libamdhip64 with the same soname as the
# system one).  Loading torch first makes this library bind to that runtime,
# so torch's allocations, streams and this library's kernels share one HIP
# runtime and one HSA instance in the process.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgeosink.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2211_00805_amd.build); there is no fallback path")

lib = C.CDLL(LIB_PATH)

c_graph = C.c_void_p
c_plan = C.c_void_p
c_stream = C.c_void_p
P_f32 = C.c_void_p     # device or host float pointers are passed as integers
P_i32 = C.c_void_p
P_f64 = C.POINTER(C.c_double)
P_i64 = C.POINTER(C.c_int64)

GS_OK = 0
STATUS = {0: "GS_OK", -1: "GS_ERR_INVALID", -2: "GS_ERR_OOM", -3: "GS_ERR_HIP", -4: "GS_ERR_NOT_CONNECTED",
          -5: "GS_ERR_SPECTRUM", -6: "GS_ERR_NONFINITE", -7: "GS_ERR_NO_DEVICE"}
GS_PLAN_AUTOTUNE = 1
GS_PLAN_NO_GRAPH = 2
GS_KERNEL_CHEBYSHEV = 0
GS_KERNEL_EULER = 1
GS_KERNEL_CLENSHAW = 2
GS_RECORD_ALL = -1
GS_MAX_K = 256

_SIGS = {
    "gs_last_error": (C.c_char_p, []),
    "gs_abi_version": (C.c_int32, []),
    "gs_graph_from_points": (C.c_int, [P_f32, C.c_int64, C.c_int32, C.c_int32, C.c_int32, c_stream,
                                       C.POINTER(c_graph)]),
    "gs_graph_from_csr": (C.c_int, [C.c_int64, C.c_int64, P_i32, P_i32, P_f32, c_stream, C.POINTER(c_graph)]),
    "gs_graph_info": (C.c_int, [c_graph, P_i64, P_i64, C.POINTER(C.c_int32), P_f64, P_f64, P_f64]),
    "gs_graph_export": (C.c_int, [c_graph, P_i32, P_i32, P_f32, P_f32]),
    "gs_graph_destroy": (None, [c_graph]),
    "gs_lambda_max": (C.c_int, [c_graph, C.c_int32, C.c_uint64, C.c_double, c_stream, P_f64]),
    "gs_cheby_coeffs": (C.c_int, [C.c_double, C.c_int32, P_f64, P_f64]),
    "gs_cheby_tail_bound": (C.c_int, [C.c_double, C.c_int32, P_f64]),
    "gs_plan_create": (C.c_int, [c_graph, C.c_int32, C.c_int32, C.c_int32, C.c_char_p, C.POINTER(c_plan)]),
    "gs_plan_set_shape": (C.c_int, [c_plan, C.c_int32, C.c_int32, C.c_int32]),
    "gs_plan_set_kernel": (C.c_int, [c_plan, C.c_int32, C.c_int32, C.c_int32]),
    "gs_plan_set_csr_hint": (C.c_int, [c_plan, C.c_int32]),
    "gs_plan_set_frontier": (C.c_int, [c_plan, C.c_int32]),
    "gs_plan_describe": (C.c_int, [c_plan, C.c_char_p, C.c_int32]),
    "gs_plan_destroy": (None, [c_plan]),
    "gs_heat_apply": (C.c_int, [c_plan, C.c_double, C.c_double, P_f32, P_f32, P_f32, c_stream]),
    "gs_heat_apply_noalloc": (C.c_int, [c_graph, C.c_double, C.c_double, C.c_int32, P_f32, P_f32, C.c_int32,
                                        c_stream]),
    "gs_sinkhorn": (C.c_int, [c_plan, C.c_double, C.c_double, P_f32, P_f32, P_f32, C.c_int32, C.c_float,
                              C.c_int32, P_f32, P_f32, P_f32, P_f64, P_f64, P_i64, c_stream]),
    "gs_sinkhorn_backward": (C.c_int, [c_plan, C.c_double, C.c_double, P_f32, P_f32, P_f32, C.c_int32, C.c_float,
                                       C.c_int32, P_f32, P_f64, P_f32, P_f32, P_f64, c_stream]),
    "gs_barycenter": (C.c_int, [c_plan, C.c_double, C.c_double, P_f32, P_f32, P_f64, C.c_int32, C.c_float,
                                P_f32, P_f32, P_f32, P_f64, P_i64, c_stream]),
    "gs_graph_heat_apply": (C.c_int, [c_graph, C.c_double, C.c_double, C.c_int32, P_f32, P_f32, P_f32, C.c_int32,
                                      c_plan, c_stream]),
    "gs_graph_sinkhorn": (C.c_int, [c_graph, C.c_double, C.c_double, C.c_int32, P_f32, P_f32, P_f32, C.c_int32,
                                    C.c_int32, C.c_float, C.c_int32, P_f32, P_f32, P_f32, P_f64, P_f64, P_i64, c_plan,
                                    c_stream]),
    "gs_graph_sinkhorn_backward": (C.c_int, [c_graph, C.c_double, C.c_double, C.c_int32, P_f32, P_f32, P_f32,
                                             C.c_int32, C.c_int32, C.c_float, C.c_int32, P_f32, P_f64, P_f32, P_f32,
                                             P_f64, c_plan, c_stream]),
    "gs_graph_barycenter": (C.c_int, [c_graph, C.c_double, C.c_double, C.c_int32, P_f32, P_f32, P_f64, C.c_int32,
                                      C.c_int32, C.c_float, P_f32, P_f32, P_f32, P_f64, P_i64, c_plan, c_stream]),
    "gs_expectation": (C.c_int, [P_f32, P_f32, C.c_int64, C.c_int32, c_stream, P_f64]),
    "gs_plan_time_step": (C.c_int, [c_plan, C.c_int32, c_stream, P_f64, P_f64]),
    "gs_stream_copy": (C.c_int, [P_f32, P_f32, C.c_int64, c_stream]),
    "gs_stream_gather": (C.c_int, [P_f32, C.c_int64, P_i32, C.c_int64, P_f32, c_stream]),
    "gs_gather_columns": (C.c_int, [P_f32, C.c_int64, C.c_int32, P_i32, C.c_int32, P_f32, c_stream]),
    "gs_accumulate_columns": (C.c_int, [P_f32, C.c_int64, C.c_int32, P_i32, C.c_int32, P_f32, c_stream]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class GeoSinkError(RuntimeError):
    """A libgeosink call returned a non-zero gs_status."""

    def __init__(self, call: str, status: int):
        self.status = status
        msg = lib.gs_last_error().decode(errors="replace")
        super().__init__(f"{call} failed with {STATUS.get(status, status)}: {msg}")


def check(call: str, status: int) -> None:
    if status != GS_OK:
        raise GeoSinkError(call, status)

"""Python binding of the C ABI (argument marshalling only).

Each function carries the name of the C entry point it calls and takes torch
tensors for device arrays (float32, contiguous, on the current HIP device) and
numpy arrays or Python scalars for host arrays.  All arithmetic of the hot path
runs in libgeosink.so's HIP kernels; torch only provides device memory and the
current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (GS_KERNEL_CHEBYSHEV, GS_KERNEL_CLENSHAW, GS_KERNEL_EULER, GS_PLAN_AUTOTUNE, GS_PLAN_NO_GRAPH, GS_RECORD_ALL,
                   GeoSinkError, check, lib)

__all__ = [
    "Graph", "Plan", "GeoSinkError", "GS_PLAN_AUTOTUNE", "GS_PLAN_NO_GRAPH", "GS_KERNEL_CHEBYSHEV", "GS_KERNEL_CLENSHAW", "GS_KERNEL_EULER",
    "GS_RECORD_ALL", "ckpt_floats",
    "gs_abi_version", "gs_graph_from_points", "gs_graph_from_csr", "gs_lambda_max", "gs_cheby_coeffs",
    "gs_cheby_tail_bound", "gs_plan_create", "gs_heat_apply", "gs_heat_apply_noalloc", "gs_sinkhorn", "gs_sinkhorn_backward",
    "gs_barycenter", "gs_expectation", "gs_gather_columns", "gs_accumulate_columns", "gs_plan_time_step", "gs_stream_copy", "gs_stream_gather", "current_stream",
]


def current_stream():
    """hipStream_t of torch's current stream on the current device."""
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor | None, name: str, numel: int | None = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _dev_min(t: torch.Tensor, name: str, numel: int):
    """As _dev, for buffers that may be larger than needed (checkpoints, records)."""
    if t is not None and isinstance(t, torch.Tensor) and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return _dev(t, name)


def gs_abi_version() -> int:
    return int(lib.gs_abi_version())


class Graph:
    """Owning wrapper of a gs_graph handle."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        n, nnz, nc = C.c_int64(), C.c_int64(), C.c_int32()
        dmax, eb, med = C.c_double(), C.c_double(), C.c_double()
        check("gs_graph_info", lib.gs_graph_info(handle, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(dmax),
                                                 C.byref(eb), C.byref(med)))
        self.n, self.nnz, self.n_components = n.value, nnz.value, nc.value
        self.deg_max, self.edge_bound, self.median = dmax.value, eb.value, med.value

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("graph was destroyed")
        return self._h

    def export(self):
        """Host copies (rowptr int32, col int32, w float32, deg float32)."""
        rp = np.empty(self.n + 1, dtype=np.int32)
        col = np.empty(max(self.nnz, 1), dtype=np.int32)
        w = np.empty(max(self.nnz, 1), dtype=np.float32)
        deg = np.empty(self.n, dtype=np.float32)
        check("gs_graph_export", lib.gs_graph_export(self.handle, rp.ctypes.data, col.ctypes.data,
                                                     w.ctypes.data, deg.ctypes.data))
        return rp, col[:self.nnz], w[:self.nnz], deg

    def destroy(self):
        if self._h is not None:
            lib.gs_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def gs_graph_from_points(X: np.ndarray, k: int, require_connected: bool = False) -> Graph:
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be (n, d)")
    h = C.c_void_p()
    check("gs_graph_from_points", lib.gs_graph_from_points(X.ctypes.data, X.shape[0], X.shape[1], int(k),
                                                           int(bool(require_connected)), current_stream(),
                                                           C.byref(h)))
    return Graph(h)


def gs_graph_from_csr(n: int, rowptr, col, w) -> Graph:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    if rowptr.shape != (n + 1,) or col.shape != w.shape:
        raise ValueError("inconsistent CSR arrays")
    h = C.c_void_p()
    check("gs_graph_from_csr", lib.gs_graph_from_csr(int(n), int(col.shape[0]), rowptr.ctypes.data,
                                                     col.ctypes.data if col.size else None,
                                                     w.ctypes.data if w.size else None, current_stream(),
                                                     C.byref(h)))
    return Graph(h)


def gs_lambda_max(graph: Graph, iters: int = 60, seed: int = 1, safety: float = 1.01) -> float:
    out = C.c_double()
    check("gs_lambda_max", lib.gs_lambda_max(graph.handle, int(iters), int(seed), float(safety), current_stream(),
                                             C.byref(out)))
    return out.value


def gs_cheby_coeffs(t: float, K: int, with_dt: bool = False):
    b = np.empty(K + 1, dtype=np.float64)
    db = np.empty(K + 1, dtype=np.float64) if with_dt else None
    check("gs_cheby_coeffs", lib.gs_cheby_coeffs(float(t), int(K), b.ctypes.data_as(_lib.P_f64),
                                                 db.ctypes.data_as(_lib.P_f64) if with_dt else None))
    return (b, db) if with_dt else b


def gs_cheby_tail_bound(t: float, K: int) -> float:
    out = C.c_double()
    check("gs_cheby_tail_bound", lib.gs_cheby_tail_bound(float(t), int(K), C.byref(out)))
    return out.value


class Plan:
    """Owning wrapper of a gs_plan handle (device workspace for (graph, K, B))."""

    def __init__(self, graph: Graph, K: int, B: int, flags: int = 0, tune_cache: str | None = None):
        h = C.c_void_p()
        check("gs_plan_create", lib.gs_plan_create(graph.handle, int(K), int(B), int(flags),
                                                   tune_cache.encode() if tune_cache else None, C.byref(h)))
        self._h = h
        self.graph, self.K, self.B, self.n = graph, int(K), int(B), graph.n

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan was destroyed")
        return self._h

    def set_shape(self, vec: int, S: int, C_: int) -> None:
        """gs_plan_set_shape: force the fused step's launch shape."""
        check("gs_plan_set_shape", lib.gs_plan_set_shape(self.handle, int(vec), int(S), int(C_)))

    def set_csr_hint(self, streamed: bool) -> None:
        """gs_plan_set_csr_hint: CSR read with non-temporal hints (streamed) or with cached loads."""
        check("gs_plan_set_csr_hint", lib.gs_plan_set_csr_hint(self.handle, int(bool(streamed))))

    def set_frontier(self, enable: bool) -> None:
        """gs_plan_set_frontier: skip rows beyond k hops of the applied supports at step k (bitwise the dense result)."""
        check("gs_plan_set_frontier", lib.gs_plan_set_frontier(self.handle, int(bool(enable))))

    def set_kernel(self, kernel: int, N: int = 0, cg_iters: int = 0) -> None:
        """gs_plan_set_kernel: Chebyshev (default) or backward-Euler (N solves of cg_iters CG steps, 0 = auto)."""
        check("gs_plan_set_kernel", lib.gs_plan_set_kernel(self.handle, int(kernel), int(N), int(cg_iters)))

    def describe(self) -> str:
        buf = C.create_string_buffer(256)
        check("gs_plan_describe", lib.gs_plan_describe(self.handle, buf, 256))
        return buf.value.decode()

    def destroy(self):
        if self._h is not None:
            lib.gs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def gs_plan_create(graph: Graph, K: int, B: int, flags: int = 0, tune_cache: str | None = None) -> Plan:
    return Plan(graph, K, B, flags, tune_cache)


def _nB(plan: Plan) -> int:
    return plan.n * plan.B


def gs_heat_apply(plan: Plan, lambda_hat: float, t: float, X: torch.Tensor, Y: torch.Tensor,
                  Ydt: torch.Tensor | None = None) -> None:
    nb = _nB(plan)
    check("gs_heat_apply", lib.gs_heat_apply(plan.handle, float(lambda_hat), float(t), _dev(X, "X", nb),
                                             _dev(Y, "Y", nb), _dev(Ydt, "Ydt", nb), current_stream()))


def gs_heat_apply_noalloc(graph: Graph, lambda_hat: float, t: float, K: int, X: torch.Tensor,
                          Y: torch.Tensor) -> None:
    """Y = p_K(L, t) X without a plan or any allocation (X, Y: n x B, B = 1 or a multiple of 4)."""
    if X.dim() == 1:
        B = 1
    elif X.dim() == 2:
        B = X.shape[1]
    else:
        raise ValueError("X must be (n,) or (n, B)")
    if X.shape[0] != graph.n or Y.numel() != X.numel():
        raise ValueError("X and Y must hold n x B floats")
    check("gs_heat_apply_noalloc", lib.gs_heat_apply_noalloc(
        graph.handle, float(lambda_hat), float(t), int(K), _dev(X, "X", X.numel()), _dev(Y, "Y", Y.numel()),
        int(B), current_stream()))


def n_checkpoints(iters: int, ckpt_every: int) -> int:
    return (int(iters) + int(ckpt_every) - 1) // int(ckpt_every)


def ckpt_floats(plan: Plan, iters: int, ckpt_every: int) -> int:
    """Floats of the ckpt buffer: checkpoints of w (n x B each), or with
    GS_RECORD_ALL the 2 * iters denominator records (n x ldp each)."""
    if int(ckpt_every) == GS_RECORD_ALL:
        ldp = 1 if plan.B == 1 else (plan.B + 3) // 4 * 4
        return 2 * int(iters) * plan.n * ldp
    return n_checkpoints(iters, ckpt_every) * plan.n * plan.B


def gs_sinkhorn(plan: Plan, lambda_hat: float, t: float, mu: torch.Tensor, nu: torch.Tensor, iters: int,
                phi: float = 1e-30, a: torch.Tensor | None = None, ckpt_every: int = 0,
                ckpt: torch.Tensor | None = None, v: torch.Tensor | None = None, w: torch.Tensor | None = None,
                want_dist: bool = True, want_marg: bool = False, want_floors: bool = False):
    """Algorithm 1 for the plan's B pairs.  Returns dict(dist, marg_err, n_floored) of host values."""
    nb = _nB(plan)
    B = plan.B
    dist = np.zeros(B, dtype=np.float64)
    marg = np.zeros(B, dtype=np.float64)
    nfl = C.c_int64(0)
    if ckpt is not None:
        _dev_min(ckpt, "ckpt", ckpt_floats(plan, iters, ckpt_every))
    check("gs_sinkhorn", lib.gs_sinkhorn(
        plan.handle, float(lambda_hat), float(t), _dev(a, "a", plan.n), _dev(mu, "mu", nb), _dev(nu, "nu", nb),
        int(iters), float(phi), int(ckpt_every), _dev(ckpt, "ckpt"), _dev(v, "v", nb), _dev(w, "w", nb),
        dist.ctypes.data_as(_lib.P_f64) if want_dist else None,
        marg.ctypes.data_as(_lib.P_f64) if want_marg else None,
        C.byref(nfl) if want_floors else None, current_stream()))
    return {"dist": dist if want_dist else None, "marg_err": marg if want_marg else None,
            "n_floored": nfl.value if want_floors else None}


def gs_sinkhorn_backward(plan: Plan, lambda_hat: float, t: float, mu: torch.Tensor, nu: torch.Tensor, iters: int,
                         ckpt_every: int, ckpt: torch.Tensor, grad_dist, phi: float = 1e-30,
                         a: torch.Tensor | None = None, grad_mu: torch.Tensor | None = None,
                         grad_nu: torch.Tensor | None = None, want_grad_t: bool = True):
    """Reverse sweep of Algorithm 1; returns the per-pair gradient in t (host) or None."""
    nb = _nB(plan)
    gd = np.ascontiguousarray(np.broadcast_to(np.asarray(grad_dist, dtype=np.float64), (plan.B,)))
    gt = np.zeros(plan.B, dtype=np.float64)
    _dev_min(ckpt, "ckpt", ckpt_floats(plan, iters, ckpt_every))
    check("gs_sinkhorn_backward", lib.gs_sinkhorn_backward(
        plan.handle, float(lambda_hat), float(t), _dev(a, "a", plan.n), _dev(mu, "mu", nb), _dev(nu, "nu", nb),
        int(iters), float(phi), int(ckpt_every), _dev(ckpt, "ckpt"), gd.ctypes.data_as(_lib.P_f64),
        _dev(grad_mu, "grad_mu", nb), _dev(grad_nu, "grad_nu", nb),
        gt.ctypes.data_as(_lib.P_f64) if want_grad_t else None, current_stream()))
    return gt if want_grad_t else None


def gs_barycenter(plan: Plan, lambda_hat: float, t: float, mus: torch.Tensor, alpha, iters: int,
                  bary: torch.Tensor, phi: float = 1e-30, a: torch.Tensor | None = None,
                  v: torch.Tensor | None = None, w: torch.Tensor | None = None, want_marg: bool = False,
                  want_floors: bool = False):
    nb = _nB(plan)
    al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    if al.shape != (plan.B,):
        raise ValueError("alpha must have B entries")
    marg = np.zeros(plan.B, dtype=np.float64)
    nfl = C.c_int64(0)
    check("gs_barycenter", lib.gs_barycenter(
        plan.handle, float(lambda_hat), float(t), _dev(a, "a", plan.n), _dev(mus, "mus", nb),
        al.ctypes.data_as(_lib.P_f64), int(iters), float(phi), _dev(bary, "bary", plan.n), _dev(v, "v", nb),
        _dev(w, "w", nb), marg.ctypes.data_as(_lib.P_f64) if want_marg else None,
        C.byref(nfl) if want_floors else None, current_stream()))
    return {"marg_err": marg if want_marg else None, "n_floored": nfl.value if want_floors else None}


# ----------------------------------------------------------------------------- graph-level forms

def _cols(graph: Graph, x: torch.Tensor, name: str) -> int:
    """Columns of an n x B (or n,) device array on the graph's nodes."""
    if x.numel() % graph.n != 0 or x.numel() == 0:
        raise ValueError(f"{name} must hold n x B floats (n = {graph.n})")
    return x.numel() // graph.n


def _plan_handle(plan: Plan | None):
    return None if plan is None else plan.handle


def gs_graph_heat_apply(graph: Graph, lambda_hat: float, t: float, K: int, X: torch.Tensor, Y: torch.Tensor,
                        Ydt: torch.Tensor | None = None, plan: Plan | None = None) -> None:
    """gs_graph_heat_apply: Y = p_K(L, t) X on the graph (B from X's size); plan None: the graph's own."""
    B = _cols(graph, X, "X")
    nb = graph.n * B
    check("gs_graph_heat_apply", lib.gs_graph_heat_apply(
        graph.handle, float(lambda_hat), float(t), int(K), _dev(X, "X", nb), _dev(Y, "Y", nb), _dev(Ydt, "Ydt", nb),
        int(B), _plan_handle(plan), current_stream()))


def gs_graph_sinkhorn(graph: Graph, lambda_hat: float, t: float, K: int, mu: torch.Tensor, nu: torch.Tensor,
                      iters: int, phi: float = 1e-30, a: torch.Tensor | None = None, ckpt_every: int = 0,
                      ckpt: torch.Tensor | None = None, v: torch.Tensor | None = None, w: torch.Tensor | None = None,
                      want_dist: bool = True, want_marg: bool = False, want_floors: bool = False,
                      plan: Plan | None = None):
    """gs_graph_sinkhorn: Algorithm 1 for the B pairs (B from mu's size); returns dict(dist, marg_err, n_floored)."""
    B = _cols(graph, mu, "mu")
    nb = graph.n * B
    dist = np.zeros(B, dtype=np.float64)
    marg = np.zeros(B, dtype=np.float64)
    nfl = C.c_int64(0)
    check("gs_graph_sinkhorn", lib.gs_graph_sinkhorn(
        graph.handle, float(lambda_hat), float(t), int(K), _dev(a, "a", graph.n), _dev(mu, "mu", nb),
        _dev(nu, "nu", nb), int(B), int(iters), float(phi), int(ckpt_every), _dev(ckpt, "ckpt"), _dev(v, "v", nb),
        _dev(w, "w", nb), dist.ctypes.data_as(_lib.P_f64) if want_dist else None,
        marg.ctypes.data_as(_lib.P_f64) if want_marg else None, C.byref(nfl) if want_floors else None,
        _plan_handle(plan), current_stream()))
    return {"dist": dist if want_dist else None, "marg_err": marg if want_marg else None,
            "n_floored": nfl.value if want_floors else None}


def gs_graph_sinkhorn_backward(graph: Graph, lambda_hat: float, t: float, K: int, mu: torch.Tensor,
                               nu: torch.Tensor, iters: int, ckpt_every: int, ckpt: torch.Tensor, grad_dist,
                               phi: float = 1e-30, a: torch.Tensor | None = None,
                               grad_mu: torch.Tensor | None = None, grad_nu: torch.Tensor | None = None,
                               want_grad_t: bool = True, plan: Plan | None = None):
    """gs_graph_sinkhorn_backward: the reverse sweep; returns the per-pair gradient in t (host) or None."""
    B = _cols(graph, mu, "mu")
    nb = graph.n * B
    gd = np.ascontiguousarray(np.broadcast_to(np.asarray(grad_dist, dtype=np.float64), (B,)))
    gt = np.zeros(B, dtype=np.float64)
    check("gs_graph_sinkhorn_backward", lib.gs_graph_sinkhorn_backward(
        graph.handle, float(lambda_hat), float(t), int(K), _dev(a, "a", graph.n), _dev(mu, "mu", nb),
        _dev(nu, "nu", nb), int(B), int(iters), float(phi), int(ckpt_every), _dev(ckpt, "ckpt"),
        gd.ctypes.data_as(_lib.P_f64), _dev(grad_mu, "grad_mu", nb), _dev(grad_nu, "grad_nu", nb),
        gt.ctypes.data_as(_lib.P_f64) if want_grad_t else None, _plan_handle(plan), current_stream()))
    return gt if want_grad_t else None


def gs_graph_barycenter(graph: Graph, lambda_hat: float, t: float, K: int, mus: torch.Tensor, alpha, iters: int,
                        bary: torch.Tensor, phi: float = 1e-30, a: torch.Tensor | None = None,
                        v: torch.Tensor | None = None, w: torch.Tensor | None = None, want_marg: bool = False,
                        want_floors: bool = False, plan: Plan | None = None):
    """gs_graph_barycenter: the barycenter of the m columns of mus (m from its size)."""
    m = _cols(graph, mus, "mus")
    nb = graph.n * m
    al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    if al.shape != (m,):
        raise ValueError("alpha must have m entries")
    marg = np.zeros(m, dtype=np.float64)
    nfl = C.c_int64(0)
    check("gs_graph_barycenter", lib.gs_graph_barycenter(
        graph.handle, float(lambda_hat), float(t), int(K), _dev(a, "a", graph.n), _dev(mus, "mus", nb),
        al.ctypes.data_as(_lib.P_f64), int(m), int(iters), float(phi), _dev(bary, "bary", graph.n),
        _dev(v, "v", nb), _dev(w, "w", nb), marg.ctypes.data_as(_lib.P_f64) if want_marg else None,
        C.byref(nfl) if want_floors else None, _plan_handle(plan), current_stream()))
    return {"marg_err": marg if want_marg else None, "n_floored": nfl.value if want_floors else None}


def gs_expectation(p: torch.Tensor, Y: torch.Tensor) -> np.ndarray:
    """sum_i p_i Y[i, :] / sum_i p_i for device p (n,) and Y (n, d) (or (n,))."""
    n = p.numel()
    d = Y.numel() // n
    if d * n != Y.numel():
        raise ValueError("Y must have n rows")
    out = np.zeros(d, dtype=np.float64)
    check("gs_expectation", lib.gs_expectation(_dev(p, "p"), _dev(Y, "Y"), n, d, current_stream(),
                                               out.ctypes.data_as(_lib.P_f64)))
    return out


def gs_gather_columns(H: torch.Tensor, cols: torch.Tensor, out: torch.Tensor) -> None:
    """out[:, b] = H[:, cols[b]] for H (n, m), cols (B,) int32 on the device, out (n, B); cols outside [0, m) give 0."""
    if H.dim() != 2 or out.dim() != 2 or out.shape[0] != H.shape[0]:
        raise ValueError("H must be (n, m) and out (n, B)")
    if cols.dtype != torch.int32 or cols.device.type != "cuda" or not cols.is_contiguous() or \
            cols.numel() != out.shape[1]:
        raise TypeError("cols must be a contiguous int32 device tensor with B entries")
    check("gs_gather_columns", lib.gs_gather_columns(
        _dev(H, "H"), H.shape[0], H.shape[1], C.c_void_p(cols.data_ptr()), out.shape[1], _dev(out, "out"),
        current_stream()))


def gs_accumulate_columns(src: torch.Tensor, cols: torch.Tensor, G: torch.Tensor) -> None:
    """G[cols[b], :] += src[:, b] for src (n, B), cols (B,) int32 on the device, G (m, n); cols outside [0, m) skipped."""
    if src.dim() != 2 or G.dim() != 2 or G.shape[1] != src.shape[0]:
        raise ValueError("src must be (n, B) and G (m, n)")
    if cols.dtype != torch.int32 or cols.device.type != "cuda" or not cols.is_contiguous() or \
            cols.numel() != src.shape[1]:
        raise TypeError("cols must be a contiguous int32 device tensor with B entries")
    check("gs_accumulate_columns", lib.gs_accumulate_columns(
        _dev(src, "src"), src.shape[0], src.shape[1], C.c_void_p(cols.data_ptr()), G.shape[0], _dev(G, "G"),
        current_stream()))


def gs_plan_time_step(plan: Plan, reps: int = 50):
    """(average ms per fused step launch, algorithmic bytes per launch)."""
    ms, by = C.c_double(), C.c_double()
    check("gs_plan_time_step", lib.gs_plan_time_step(plan.handle, int(reps), current_stream(), C.byref(ms),
                                                     C.byref(by)))
    return ms.value, by.value


def gs_stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    if src.numel() != dst.numel():
        raise ValueError("src and dst sizes differ")
    check("gs_stream_copy", lib.gs_stream_copy(_dev(src, "src"), _dev(dst, "dst"), src.numel(), current_stream()))


def gs_stream_gather(X: torch.Tensor, idx: torch.Tensor, out: torch.Tensor) -> None:
    """Sum runs of 32 gathered 128-byte rows X[idx] (X: (n, 32) float32, idx: int32) into out."""
    if X.dim() != 2 or X.shape[1] != 32:
        raise ValueError("X must be (n, 32)")
    if idx.dtype != torch.int32 or idx.device.type != "cuda" or not idx.is_contiguous():
        raise TypeError("idx must be a contiguous int32 device tensor")
    m = idx.numel()
    check("gs_stream_gather", lib.gs_stream_gather(_dev(X, "X"), X.shape[0], C.c_void_p(idx.data_ptr()), m,
                                                   _dev(out, "out", (m + 31) // 32 * 32), current_stream()))

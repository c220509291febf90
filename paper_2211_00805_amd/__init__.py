"""Geodesic Sinkhorn on MI355X (gfx950): C-ABI library libgeosink.so + thin binding.

The binding modules are loaded on first attribute access, so that the build
script can run before the library exists; any use of the product path then
fails loudly (ImportError) when libgeosink.so has not been built.
"""
from __future__ import annotations

import importlib

_API = ("Graph", "Plan", "GeoSinkError", "GS_PLAN_AUTOTUNE", "GS_PLAN_NO_GRAPH", "GS_KERNEL_CHEBYSHEV", "GS_KERNEL_CLENSHAW",
        "GS_KERNEL_EULER", "GS_RECORD_ALL", "ckpt_floats", "gs_abi_version",
        "gs_graph_from_points", "gs_graph_from_csr", "gs_lambda_max", "gs_cheby_coeffs", "gs_cheby_tail_bound",
        "gs_plan_create", "gs_heat_apply", "gs_heat_apply_noalloc", "gs_sinkhorn", "gs_sinkhorn_backward", "gs_barycenter",
        "gs_graph_heat_apply", "gs_graph_sinkhorn", "gs_graph_sinkhorn_backward", "gs_graph_barycenter",
        "gs_expectation", "gs_gather_columns", "gs_accumulate_columns", "gs_plan_time_step", "gs_stream_copy", "gs_stream_gather", "current_stream", "n_checkpoints")
_AUTOGRAD = ("GeoSinkhornDistance", "geodesic_sinkhorn_distance")
_FAMILIES = ("family_barycenter", "barycentric_distance", "expected_barycenter_effect")
_PAIRWISE = ("distance_matrix", "nn_scores", "precision_at_k", "pair_list")

__all__ = list(_API + _AUTOGRAD + _FAMILIES + _PAIRWISE)


def __getattr__(name):
    if name in _API:
        return getattr(importlib.import_module(".api", __name__), name)
    if name in _AUTOGRAD:
        return getattr(importlib.import_module(".autograd", __name__), name)
    if name in _FAMILIES:
        return getattr(importlib.import_module(".families", __name__), name)
    if name in _PAIRWISE:
        return getattr(importlib.import_module(".pairwise", __name__), name)
    raise AttributeError(name)

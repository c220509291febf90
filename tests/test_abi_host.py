"""Host-side checks of the C-ABI library (no GPU needed, no device compute).

The library loads, exports every entry point declared in include/geosink.h,
computes the Chebyshev coefficients on the host like the oracle, and rejects
bad arguments before touching HIP.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geosink.h")
LIB = os.path.join(ROOT, "paper_2211_00805_amd", "libgeosink.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgeosink.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["gs_graph_from_points", "gs_graph_from_csr", "gs_lambda_max", "gs_cheby_coeffs", "gs_heat_apply",
                 "gs_sinkhorn", "gs_sinkhorn_backward", "gs_barycenter", "gs_plan_create"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(gs_[a-z_]+)$", out, flags=re.M))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    lib = C.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_binding_covers_every_symbol():
    from paper_2211_00805_amd import _lib
    assert set(declared_symbols()) == set(_lib.EXPORTED)


@pytest.mark.parametrize("t,K", [(0.5, 30), (1.0, 20), (2.0, 50), (8.0, 30), (1e-3, 10), (40.0, 120)])
def test_coefficients_match_oracle(t, K):
    from oracle import heat
    from paper_2211_00805_amd import gs_cheby_coeffs, gs_cheby_tail_bound
    b, db = gs_cheby_coeffs(t, K, with_dt=True)
    np.testing.assert_allclose(b, heat.cheb_coeffs(t, K), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(db, heat.cheb_coeffs_dt(t, K), rtol=1e-10, atol=1e-15)
    assert gs_cheby_tail_bound(t, K) == pytest.approx(heat.tail_bound(t, K), rel=1e-9, abs=1e-300)


def test_coefficients_at_t_zero_are_identity():
    from paper_2211_00805_amd import gs_cheby_coeffs
    b = gs_cheby_coeffs(0.0, 6)
    assert b[0] == 2.0 and np.all(b[1:] == 0.0)


def test_validation_rejects_before_any_device_call():
    from paper_2211_00805_amd._lib import lib
    h = C.c_void_p()
    assert lib.gs_plan_create(None, 10, 4, 0, None, C.byref(h)) == -1
    assert b"graph is NULL" in lib.gs_last_error()
    assert lib.gs_cheby_coeffs(1.0, -1, None, None) == -1
    b = np.zeros(4)
    assert lib.gs_cheby_coeffs(float("nan"), 3, b.ctypes.data_as(C.POINTER(C.c_double)), None) == -1
    assert lib.gs_cheby_coeffs(1.0, 100000, b.ctypes.data_as(C.POINTER(C.c_double)), None) == -1
    # CSR checks run on the host before any HIP call
    rp = np.array([0, 1, 1], dtype=np.int32)
    col = np.array([1], dtype=np.int32)
    w = np.array([1.0], dtype=np.float32)
    assert lib.gs_graph_from_csr(2, 1, rp.ctypes.data, col.ctypes.data, w.ctypes.data, None, C.byref(h)) == -1
    assert b"symmetric" in lib.gs_last_error()
    rp = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 0], dtype=np.int32)
    w = np.array([1.0, 1.0], dtype=np.float32)
    assert lib.gs_graph_from_csr(2, 2, rp.ctypes.data, col.ctypes.data, w.ctypes.data, None, C.byref(h)) == -1
    assert b"self loop" in lib.gs_last_error()
    X = np.array([[0.0], [np.inf], [1.0]], dtype=np.float32)
    assert lib.gs_graph_from_points(X.ctypes.data, 3, 1, 1, 0, None, C.byref(h)) == -6
    assert lib.gs_sinkhorn(None, 2.0, 1.0, None, None, None, 1, 1e-30, 0, None, None, None, None, None, None,
                           None) == -1
    assert lib.gs_heat_apply(None, 2.0, 1.0, None, None, None, None) == -1
    assert lib.gs_plan_set_kernel(None, 1, 4, 0) == -1
    assert b"plan is NULL" in lib.gs_last_error()
    assert lib.gs_expectation(None, None, 10, 1, None, None) == -1
    ms, by = C.c_double(), C.c_double()
    assert lib.gs_plan_time_step(None, 10, None, C.byref(ms), C.byref(by)) == -1
    assert lib.gs_stream_copy(None, None, 4, None) == -1
    assert lib.gs_stream_gather(None, 10, None, 4, None, None) == -1
    assert lib.gs_accumulate_columns(None, 10, 4, None, 2, None, None) == -1
    assert b"NULL" in lib.gs_last_error()
    assert lib.gs_plan_set_csr_hint(None, 1) == -1
    assert b"plan is NULL" in lib.gs_last_error()
    assert lib.gs_plan_set_frontier(None, 1) == -1
    assert b"plan is NULL" in lib.gs_last_error()
    assert lib.gs_graph_heat_apply(None, 2.0, 1.0, 10, None, None, None, 4, None, None) == -1
    assert b"graph is NULL" in lib.gs_last_error()
    assert lib.gs_graph_sinkhorn(None, 2.0, 1.0, 10, None, None, None, 4, 5, 1e-30, 0, None, None, None, None,
                                 None, None, None, None) == -1
    assert b"graph is NULL" in lib.gs_last_error()
    assert lib.gs_graph_sinkhorn_backward(None, 2.0, 1.0, 10, None, None, None, 4, 5, 1e-30, 1, None, None, None,
                                          None, None, None, None) == -1
    assert b"graph is NULL" in lib.gs_last_error()
    assert lib.gs_graph_barycenter(None, 2.0, 1.0, 10, None, None, None, 4, 5, 1e-30, None, None, None, None, None,
                                   None, None) == -1
    assert b"graph is NULL" in lib.gs_last_error()
    assert lib.gs_heat_apply_noalloc(None, 2.0, 1.0, 10, None, None, 4, None) == -1
    assert b"graph is NULL" in lib.gs_last_error()


def test_abi_version():
    from paper_2211_00805_amd import gs_abi_version
    assert gs_abi_version() == 2

"""The entry point that allocates nothing, gs_heat_apply_noalloc, against gs_heat_apply.

Both compute Y = p_K(L, t) X (Sec. "Chebyshev Polynomials") with the same
accumulating step kernel and schedule; the no-allocation form keeps its
Chebyshev buffers in the library's fixed device array instead of a plan's
workspace.  Where the plan takes no long-row blocks (no row above the
threshold) and uses the same default launch shape, the two are bitwise equal;
with hub rows (the plan's long-row blocks sum in another order) they agree to
the heat-application tolerance, and both match the float64 oracle.  Two calls
in a row, the second on a smaller input; sizes beyond the array are refused;
the call is captured into a hipGraph and replayed.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import heat
from gpu_common import csr_laplacian, heat_tol, lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


def plan_apply(gs, g, lam, t, K, x):
    n, B = x.shape
    plan = gs.Plan(g, K, B)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    torch.cuda.synchronize()
    return to_host(Y).reshape(n, B), plan.describe()


def test_two_calls_bitwise_equal_to_plan_form(gs):
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    n = 2000
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    for B, K, t in ((32, 20, 1.0), (4, 7, 2.0)):   # the second call smaller
        x = synth.random_dense_like(n, B, np.random.default_rng(B + K))
        Y = torch.full((n, B), float("nan"), device="cuda")
        gs.gs_heat_apply_noalloc(g, lam, t, K, to_dev(x), Y)
        torch.cuda.synchronize()
        got = to_host(Y)
        want, desc = plan_apply(gs, g, lam, t, K, x)
        assert np.array_equal(got, want), (B, K, desc, np.abs(got - want).max())
        ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
        assert np.abs(got - ref).max() <= heat_tol(K, np.abs(x).max())


def test_single_column_and_hub_rows(gs):
    n, K, t = 6000, 9, 1.5
    arrs = synth.random_local_graph(n, 6, 300, np.random.default_rng(21), hubs=4, hub_degree=2900)
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    for B in (8, 1):
        x = synth.random_dense_like(n, B, np.random.default_rng(30 + B))
        Y = torch.empty((n, B), device="cuda")
        gs.gs_heat_apply_noalloc(g, lam, t, K, to_dev(x), Y)
        torch.cuda.synchronize()
        got = to_host(Y)
        want, _ = plan_apply(gs, g, lam, t, K, x)
        tol = heat_tol(K, np.abs(x).max())
        assert np.abs(got - want).max() <= tol
        assert np.abs(got - heat.heat_apply(L, lam, t, K, x.astype(np.float64))).max() <= tol


def test_sizes_beyond_the_array_are_refused(gs):
    n = 1_100_000   # n * 4 > GS_NOALLOC_MAX_NB = 4 * 2^20
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    x = torch.zeros((n, 4), device="cuda")
    y = torch.zeros((n, 4), device="cuda")
    with pytest.raises(gs.GeoSinkError) as e:
        gs.gs_heat_apply_noalloc(g, 4.0, 1.0, 10, x, y)
    assert e.value.status == -1 and "GS_NOALLOC_MAX_NB" in str(e.value)
    x1 = torch.ones(n, device="cuda")
    y1 = torch.empty(n, device="cuda")
    gs.gs_heat_apply_noalloc(g, 4.0, 1.0, 10, x1, y1)   # B = 1 fits
    torch.cuda.synchronize()
    p0 = float(np.sum(heat.cheb_coeffs(1.0, 10)[1:] * (-1.0) ** np.arange(1, 11)) + 0.5 * heat.cheb_coeffs(1.0, 10)[0])
    assert np.allclose(to_host(y1), p0, rtol=1e-6)   # L 1 = 0: p_K 1 = p_K(0) 1
    x3 = torch.zeros((1000, 3), device="cuda")
    g3 = gs.gs_graph_from_csr(1000, *synth.cycle_graph(1000))
    with pytest.raises(gs.GeoSinkError):
        gs.gs_heat_apply_noalloc(g3, 4.0, 1.0, 10, x3, torch.zeros_like(x3))


def test_captured_into_a_hip_graph_and_replayed(gs):
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    n, B, K, t = 2000, 16, 20, 1.0
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = to_dev(synth.random_dense_like(n, B, np.random.default_rng(3)).reshape(n, B))
    y_eager = torch.empty((n, B), device="cuda")
    gs.gs_heat_apply_noalloc(g, lam, t, K, x, y_eager)   # first call on the device: outside capture
    torch.cuda.synchronize()
    y = torch.empty((n, B), device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            gs.gs_heat_apply_noalloc(g, lam, t, K, x, y)
    torch.cuda.synchronize()
    for r in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), r
        # eager work between replays: the plan form on the same device
        plan_apply(gs, g, lam, t, K, to_host(x))

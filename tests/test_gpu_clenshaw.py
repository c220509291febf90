"""GPU parity of the Clenshaw form of the heat kernel (GS_KERNEL_CLENSHAW).

p_K(L, t) X = b_0/2 X + sum_k b_k T_k(y) X (Sec. "Chebyshev Polynomials") is
evaluated by Clenshaw's backward recurrence u_k = 2 y u_{k+1} - u_{k+2} + b_k X,
result y u_1 - u_2 + (b_0/2) X, one fused sparse product per step (K products,
as the accumulating form).  Everything is compared with the float64 oracle,
which evaluates the forward three-term recurrence with the same coefficients:
heat applications element by element (every launch shape, K = 1, 2, 3, 20,
ragged widths, hub rows, n = 1M on sampled columns), Algorithm 1 (distances
and plans), the barycenter and the reverse sweep (whose time-derivative
applications keep the accumulating form, which has the second accumulator).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms, heat
from oracle import sinkhorn as osk
from gpu_common import csr_laplacian, heat_tol, lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def swiss():
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    return arrs, L


def clen_plan(gs, g, K, B, flags=0):
    plan = gs.Plan(g, K, B, flags=flags)
    plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
    assert "kernel=clenshaw" in plan.describe()
    return plan


def _shapes(B):
    if B == 1:
        return [(1, S, 1) for S in (2, 4, 8, 16, 32, 64)]
    ldp = (B + 3) // 4 * 4
    return [(4, S, C) for C in (1, 2, 4, 8, 16, 32, 64) if C == 1 or C // 2 < ldp // 4
            for S in (1, 2, 4, 8, 16) if S * C <= 64]


@pytest.mark.parametrize("B", [1, 3, 32, 35])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 20])
def test_clenshaw_heat_apply(gs, swiss, B, K):
    arrs, L = swiss
    n, t = 2000, 1.0
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = synth.random_dense_like(n, B, np.random.default_rng(B * 10 + K))
    plan = clen_plan(gs, g, K, B)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    err = np.abs(to_host(Y).reshape(n, B) - ref).max()
    assert err <= heat_tol(K, np.abs(x).max()), (err, plan.describe())


@pytest.mark.parametrize("B", [1, 10, 32])
def test_clenshaw_every_launch_shape_and_hub_rows(gs, B):
    """Every launch shape, direct launches and captured graphs, on a graph with
    hub rows of 2900 nonzeros (the long-row blocks)."""
    n, K, t = 6000, 9, 1.5
    arrs = synth.random_local_graph(n, 6, 300, np.random.default_rng(21), hubs=4, hub_degree=2900)
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    x = synth.random_dense_like(n, B, np.random.default_rng(22))
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    for flags in (0, gs.GS_PLAN_NO_GRAPH):
        plan = clen_plan(gs, g, K, B, flags)
        Y = torch.empty(n * B, device="cuda")
        for shape in _shapes(B):
            plan.set_shape(*shape)
            plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
            gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
            err = np.abs(to_host(Y).reshape(n, B) - ref).max()
            assert err <= heat_tol(K, np.abs(x).max()), (shape, err)


def test_clenshaw_time_derivative_keeps_accumulators(gs, swiss):
    """Y and dY/dt together: the time derivative needs the second accumulator,
    so this application runs in the accumulating form under either kernel."""
    arrs, L = swiss
    n, K, t, B = 2000, 30, 2.0, 8
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = synth.random_dense_like(n, B, np.random.default_rng(5))
    plan = clen_plan(gs, g, K, B)
    Y = torch.empty(n * B, device="cuda")
    Yd = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y, Yd)
    tol = heat_tol(K, np.abs(x).max())
    assert np.abs(to_host(Y).reshape(n, B) - heat.heat_apply(L, lam, t, K, x.astype(np.float64))).max() <= tol
    assert np.abs(to_host(Yd).reshape(n, B) - heat.heat_apply_dt(L, lam, t, K, x.astype(np.float64))).max() <= 2 * tol


def test_clenshaw_cycle_one_million_nodes(gs):
    """n = 1M cycle, K = 50: the exact polynomial at the Fourier eigenvalues."""
    n, K, t, lam, B = 1_000_000, 50, 2.0, 4.0, 4
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    x = synth.random_dense_like(n, B, np.random.default_rng(3))
    plan = clen_plan(gs, g, K, B)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = closed_forms.cycle_heat_apply(n, lam, t, K, x.astype(np.float64))
    assert np.abs(to_host(Y).reshape(n, B) - ref).max() <= heat_tol(K, np.abs(x).max())


def test_clenshaw_sinkhorn_swiss_roll(gs, swiss):
    """Algorithm 1 on the Swiss-roll workload (K = 20, t = 1, J = 200) through the Clenshaw kernel."""
    arrs, L = swiss
    n, K, t, J = 2000, 20, 1.0, 200
    rng = np.random.default_rng(synth.seed_for(1, 2))
    mu = synth.uniform_on_random_nodes(n, 500, rng)
    nu = synth.uniform_on_random_nodes(n, 500, rng)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = clen_plan(gs, g, K, 1)
    v = torch.empty(n, device="cuda")
    w = torch.empty(n, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, v=v, w=w, want_floors=True)
    assert np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)
    r = osk.row_marginal(L, lam, t, K, to_host(v), to_host(w))
    rr = osk.row_marginal(L, lam, t, K, ref["v"], ref["w"])
    assert np.abs(r - rr).sum() <= 1e-6
    assert out["n_floored"] == ref["n_floored"] == 0


def test_clenshaw_barycenter(gs):
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    n, m, K, t, J = X.shape[0], 8, 20, 2.0, 40
    H, _ = synth.loguniform_support_histograms(n, m, 30, 1500, 0.5, np.random.default_rng(3))
    lam = lam_hat_of(L)
    alpha = np.full(m, 1.0 / m)
    ref = osk.barycenter(L, lam, t, K, H.astype(np.float64), alpha, J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = clen_plan(gs, g, K, m)
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, to_dev(H), alpha, J, bary)
    assert np.abs(to_host(bary) - ref["p"]).sum() <= 1e-6


@pytest.mark.parametrize("ce", [5, -1])
def test_clenshaw_reverse_sweep(gs, ce):
    """Gradients in mu, nu and t through the Clenshaw kernel (records or checkpoints)
    against the oracle's reverse mode."""
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    n, K, t, J, B = X.shape[0], 15, 2.0, 12, 4
    rng = np.random.default_rng(8)
    pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in (0, 2, 4, 6)]
    mu = np.stack([p[0] for p in pairs], axis=1)
    nu = np.stack([p[1] for p in pairs], axis=1)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = clen_plan(gs, g, K, B)
    ce = gs.GS_RECORD_ALL if ce < 0 else ce
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    mud, nud = to_dev(mu), to_dev(nu)
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=ce, ckpt=ckpt)
    assert np.all(np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t))
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ckpt, np.ones(B), grad_mu=gmu, grad_nu=gnu)
    for got, want, h in ((gmu, ref["dmu"], mu), (gnu, ref["dnu"], nu)):
        G = to_host(got).reshape(n, B)
        s = h > 0
        rel = np.linalg.norm(G[s] - want[s]) / np.linalg.norm(want[s])
        assert rel <= 1e-4, rel
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)


def test_clenshaw_one_million_nodes_sampled_columns(gs):
    """n = 1M random local graph with hub rows (18.4M nonzeros), B = 32, K = 50,
    the autotuned launch: three columns against the oracle."""
    n, K, t, B = 1_000_000, 50, 2.0, 32
    arrs = synth.local_graph_1m()
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    x = synth.random_dense_like(n, B, np.random.default_rng(16))
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE)
    plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    cols = [0, 19, 31]
    ref = heat.heat_apply(L, lam, t, K, x[:, cols].astype(np.float64))
    err = np.abs(to_host(Y).reshape(n, B)[:, cols] - ref).max()
    assert err <= heat_tol(K, np.abs(x).max()), (err, plan.describe())


@pytest.mark.parametrize("K", [1, 2, 3])
def test_clenshaw_sinkhorn_smallest_degrees_with_vertex_weights(gs, K):
    """Algorithm 1 with vertex weights through the Clenshaw kernel at K = 1, 2, 3,
    where the first and last products coincide or touch (the scaling epilogue
    on product 1, the folded u_K term on the last): distances and plans."""
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    n, t, J, B = 2000, 1.0, 30, 4
    rng = np.random.default_rng(40 + K)
    mu = np.stack([synth.uniform_on_random_nodes(n, 300, rng) for _ in range(B)], axis=1)
    nu = np.stack([synth.uniform_on_random_nodes(n, 300, rng) for _ in range(B)], axis=1)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, a=a.astype(np.float64))
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = clen_plan(gs, g, K, B)
    v = torch.empty(n * B, device="cuda")
    w = torch.empty(n * B, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, a=to_dev(a), v=v, w=w, want_floors=True)
    assert out["n_floored"] == ref["n_floored"]
    assert np.all(np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)), (out["dist"], ref["D"])
    r = osk.row_marginal(L, lam, t, K, to_host(v).reshape(n, B), to_host(w).reshape(n, B), a.astype(np.float64))
    rr = osk.row_marginal(L, lam, t, K, ref["v"], ref["w"], a.astype(np.float64))
    assert np.abs(r - rr).sum(axis=0).max() <= 1e-6

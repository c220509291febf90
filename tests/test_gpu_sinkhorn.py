"""GPU parity of Algorithm 1 (Geodesic Sinkhorn) against the float64 oracle.

Tolerances: distances |dD| <= 1e-5 max(|D_ref|, 4t); plans: the row marginal
a v p_K(a w) of the GPU's (v, w) and of the oracle's (v, w), both evaluated
with the oracle's float64 operator, within 1e-6 in L1.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import sinkhorn as osk
from gpu_common import lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


def dist_ok(D, Dref, t):
    return np.abs(D - Dref) <= 1e-5 * np.maximum(np.abs(Dref), 4 * t)


def plan_l1(L, lam, t, K, v, w, vr, wr, a=None):
    r = osk.row_marginal(L, lam, t, K, v, w, a)
    rr = osk.row_marginal(L, lam, t, K, vr, wr, a)
    return np.abs(r - rr).sum(axis=0)


@pytest.fixture(scope="module")
def swiss():
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    return arrs, L


def test_swiss_roll_workload(gs, swiss):
    """n = 2000, k = 10, K = 20, t = 1, two uniform histograms on 500 random nodes, 200 iterations."""
    arrs, L = swiss
    n, K, t, J = 2000, 20, 1.0, 200
    rng = np.random.default_rng(synth.seed_for(1, 2))
    mu = synth.uniform_on_random_nodes(n, 500, rng)
    nu = synth.uniform_on_random_nodes(n, 500, rng)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    v = torch.empty(n, device="cuda")
    w = torch.empty(n, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, v=v, w=w, want_marg=True, want_floors=True)
    assert dist_ok(out["dist"], ref["D"], t).all(), (out["dist"], ref["D"])
    l1 = plan_l1(L, lam, t, K, to_host(v), to_host(w), ref["v"], ref["w"])
    assert l1.max() <= 1e-6, l1
    assert out["n_floored"] == ref["n_floored"] == 0
    assert out["marg_err"][0] == pytest.approx(ref["marg_row"][0], rel=1e-2, abs=1e-7)


@pytest.mark.parametrize("t", [0.5, 2.0, 8.0])
def test_cluster_curve_pair(gs, t):
    """Reduced-size twin of the R^50 cluster-curve workload: 20 clusters x 400, k = 15, K = 30,
    Dirichlet(1) on clusters 0-3 vs 4-7."""
    X, labels = synth.clusters_on_curve(20, 400, dim=50, sigma=0.1, workload=2)
    arrs, L, info, A = oracle_csr(X, 15)
    assert info["n_components"] == 1
    n, K, J = X.shape[0], 30, 100
    rng = np.random.default_rng(synth.seed_for(2, 2))
    mu, nu = synth.cluster_block_pair(labels, 0, 4, 1.0, rng)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    v = torch.empty(n, device="cuda")
    w = torch.empty(n, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, v=v, w=w, want_floors=True)
    assert dist_ok(out["dist"], ref["D"], t).all(), (out["dist"], ref["D"])
    assert plan_l1(L, lam, t, K, to_host(v), to_host(w), ref["v"], ref["w"]).max() <= 1e-6
    assert out["n_floored"] == ref["n_floored"]


def test_batched_pairs_match_per_pair_oracle(gs):
    """B = 12 pairs with uneven supports in one multi-RHS launch (ragged padding to 12)."""
    X, labels = synth.clusters_on_curve(12, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    n, K, t, J, B = X.shape[0], 30, 2.0, 60, 12
    rng = np.random.default_rng(33)
    H, sizes = synth.loguniform_support_histograms(n, 2 * B, 50, 2000, 0.5, rng)
    mu, nu = H[:, :B].copy(), H[:, B:].copy()
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE)
    v = torch.empty(n * B, device="cuda")
    w = torch.empty(n * B, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, v=v, w=w)
    assert dist_ok(out["dist"], ref["D"], t).all(), (out["dist"] - ref["D"])
    l1 = plan_l1(L, lam, t, K, to_host(v).reshape(n, B), to_host(w).reshape(n, B), ref["v"], ref["w"])
    assert l1.max() <= 1e-6, l1


def test_vertex_weights(gs, swiss):
    arrs, L = swiss
    n, K, t, J = 2000, 20, 1.0, 50
    rng = np.random.default_rng(44)
    a = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    mu = synth.uniform_on_random_nodes(n, 300, rng)
    nu = synth.uniform_on_random_nodes(n, 300, rng)
    mu64, nu64, a64 = mu.astype(np.float64), nu.astype(np.float64), a.astype(np.float64)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn(L, lam, t, K, mu64, nu64, J, a=a64)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    v = torch.empty(n, device="cuda")
    w = torch.empty(n, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, a=to_dev(a), v=v, w=w)
    assert dist_ok(out["dist"], ref["D"], t).all(), (out["dist"], ref["D"])
    assert plan_l1(L, lam, t, K, to_host(v), to_host(w), ref["v"], ref["w"], a64).max() <= 1e-6


def test_floors_counted_like_oracle(gs):
    """Supports farther apart than K hops: every denominator on mu's support is floored."""
    n, K, t, J = 400, 6, 1.0, 3
    arrs = synth.cycle_graph(n)
    from gpu_common import csr_laplacian
    L = csr_laplacian(n, arrs)
    mu = np.zeros(n, dtype=np.float32)
    mu[:5] = 0.2
    nu = np.zeros(n, dtype=np.float32)
    nu[200:205] = 0.2
    ref = osk.sinkhorn(L, 4.0, t, K, mu.astype(np.float64), nu.astype(np.float64), J, phi=1e-30)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    out = gs.gs_sinkhorn(plan, 4.0, t, to_dev(mu), to_dev(nu), J, want_floors=True)
    assert ref["n_floored"] > 0
    assert out["n_floored"] == ref["n_floored"]


def test_run_to_run_bitwise_determinism(gs, swiss):
    arrs, L = swiss
    n, K, t, J, B = 2000, 20, 1.0, 30, 8
    rng = np.random.default_rng(55)
    H, _ = synth.loguniform_support_histograms(n, 2 * B, 20, 800, 1.0, rng)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    lam = lam_hat_of(L)
    res = []
    for _ in range(2):
        v = torch.empty(n * B, device="cuda")
        out = gs.gs_sinkhorn(plan, lam, t, to_dev(H[:, :B]), to_dev(H[:, B:]), J, v=v)
        res.append((out["dist"].copy(), v.clone()))
    assert np.array_equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1], res[1][1])

"""GPU parity of the graph build, lambda_hat estimate and heat application.

The library's kNN graph is compared with the oracle's (structure bit-exact,
weights to float32 rounding).  Heat applications run on the oracle's graph
(float32 weights given to both sides through gs_graph_from_csr) and are
compared element by element with the oracle's float64 recurrence, over every
launch shape, several widths B (with ragged padding) and node counts that
leave ragged row tiles; at full size (n = 1M) against the FFT closed form of
the cycle and against the oracle on a kNN-sized random graph.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms, heat, spectrum
from gpu_common import csr_laplacian, heat_tol, lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def swiss():
    """The Swiss-roll workload: n = 2000 in R^10, k = 10."""
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    return X, arrs, L, info, A


def test_graph_from_points_matches_oracle(gs, swiss):
    X, (rp, col, w32), L, info, A = swiss
    g = gs.gs_graph_from_points(X, 10)
    grp, gcol, gw, gdeg = g.export()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_allclose(gw, A.data, rtol=2 * 2.0 ** -24, atol=0)
    assert g.median == pytest.approx(info["median"], rel=1e-12)
    assert g.n_components == info["n_components"] == 1
    np.testing.assert_allclose(gdeg, np.asarray(A.sum(axis=1)).ravel(), rtol=1e-6)
    assert g.edge_bound >= spectrum.lambda_max(L)


def test_graph_from_points_clusters_r50(gs):
    X, labels = synth.clusters_on_curve(10, 600, dim=50, sigma=0.1, workload=2)
    (rp, col, w32), L, info, A = oracle_csr(X, 15)
    g = gs.gs_graph_from_points(X, 15)
    grp, gcol, gw, _ = g.export()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_allclose(gw, A.data, rtol=2 * 2.0 ** -24, atol=0)
    assert g.n_components == info["n_components"]


@pytest.mark.parametrize("shape,k", [((32, 32), 10), ((10, 10, 10), 20), ((10, 10, 10), 27)])
def test_graph_from_points_exact_ties_on_integer_lattices(gs, shape, k):
    """Integer lattices (d = 2, 3): every float32 Gram distance is exact, so
    neighbours tie in whole shells (4, 8, 12 or 24 points at one distance);
    the graph must follow the lower-id rule exactly as the oracle does, also
    where a shell straddles the k-th place."""
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    X = np.stack([g.ravel() for g in grids], axis=1).astype(np.float32)
    (rp, col, w32), L, info, A = oracle_csr(X, k)
    g = gs.gs_graph_from_points(X, k)
    grp, gcol, gw, _ = g.export()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_allclose(gw, A.data, rtol=2 * 2.0 ** -24, atol=0)
    assert g.median == pytest.approx(info["median"], rel=1e-12)


def test_graph_from_points_with_duplicate_points(gs):
    """Some duplicated points (distance 0, weight exp(0) = 1, ties to the lower
    id) match the oracle; a cloud whose median neighbour distance is 0 (every
    point repeated 12 times, k = 10) is refused, since exp(-d^2 / m^2) is then
    undefined."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 5)).astype(np.float32)
    X = np.concatenate([X, X[rng.choice(300, 40, replace=False)]])
    (rp, col, w32), L, info, A = oracle_csr(X, 8)
    assert info["median"] > 0 and np.any(info["directed_dist"] == 0)
    g = gs.gs_graph_from_points(X, 8)
    grp, gcol, gw, _ = g.export()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_allclose(gw, A.data, rtol=2 * 2.0 ** -24, atol=0)
    dup = np.repeat(rng.standard_normal((50, 5)).astype(np.float32), 12, axis=0)
    with pytest.raises(gs.GeoSinkError) as e:
        gs.gs_graph_from_points(dup, 10)
    assert e.value.status == -1 and "median" in str(e.value)


@pytest.mark.parametrize("n,k,d", [(2, 1, 3), (20, 19, 3), (131, 32, 7)])
def test_graph_from_points_tiny_and_complete(gs, n, k, d):
    """Fewer points than one 128-point tile, k = n - 1 (the complete graph:
    fewer other points than the k + 8 candidate slots), the largest k, an
    odd dimension: the same CSR as the oracle."""
    X = np.random.default_rng(n + k).standard_normal((n, d)).astype(np.float32)
    (rp, col, w32), L, info, A = oracle_csr(X, k)
    g = gs.gs_graph_from_points(X, k)
    grp, gcol, gw, _ = g.export()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_allclose(gw, A.data, rtol=2 * 2.0 ** -24, atol=0)
    if k == n - 1:
        assert len(gcol) == n * (n - 1)


def test_lambda_max_bounds(gs, swiss):
    X, arrs, L, info, A = swiss
    g = gs.gs_graph_from_csr(2000, *arrs)
    lmax = spectrum.lambda_max(L)
    lam = gs.gs_lambda_max(g, iters=60, seed=7, safety=1.01)
    assert lmax <= lam <= g.edge_bound * (1 + 1e-12)
    assert lam <= 1.02 * lmax


@pytest.mark.parametrize("B", [1, 3, 4, 8, 32, 64, 100])
@pytest.mark.parametrize("K", [1, 2, 3, 20])
def test_heat_apply_default_shape(gs, swiss, B, K):
    X, arrs, L, info, A = swiss
    n = 2000
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    t = 1.0
    rng = np.random.default_rng(B * 100 + K)
    x = synth.random_dense_like(n, B, rng)
    plan = gs.Plan(g, K, B)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    err = np.abs(to_host(Y).reshape(n, B) - ref).max()
    assert err <= heat_tol(K, np.abs(x).max()), (err, plan.describe())


def _shapes(B):
    """Every supported shape: C column lanes need not divide the padded row
    (lanes past it idle), but must be 1 or below twice its float4 groups."""
    if B == 1:
        return [(1, S, 1) for S in (2, 4, 8, 16, 32, 64)]
    ldp = (B + 3) // 4 * 4
    out = []
    for C in (1, 2, 4, 8, 16, 32, 64):
        if C > 1 and C // 2 >= ldp // 4:
            continue
        for S in (1, 2, 4, 8, 16):
            if S * C <= 64:
                out.append((4, S, C))
    return out


@pytest.mark.parametrize("B", [1, 8, 10, 32, 35, 64])
def test_heat_apply_every_launch_shape(gs, swiss, B):
    X, arrs, L, info, A = swiss
    n, K, t = 2000, 5, 2.0
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = synth.random_dense_like(n, B, np.random.default_rng(B))
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    plan = gs.Plan(g, K, B)
    xd = to_dev(x)
    Y = torch.empty(n * B, device="cuda")
    for shape in _shapes(B):
        plan.set_shape(*shape)
        outs = []
        for streamed in (True, False):   # CSR loads non-temporal or cached: bitwise the same
            plan.set_csr_hint(streamed)
            gs.gs_heat_apply(plan, lam, t, xd, Y)
            outs.append(to_host(Y).reshape(n, B))
            err = np.abs(outs[-1] - ref).max()
            assert err <= heat_tol(K, np.abs(x).max()), (shape, streamed, err)
        assert np.array_equal(outs[0], outs[1]), shape


@pytest.mark.parametrize("B", [1, 10, 32])
def test_heat_apply_rows_of_very_high_degree(gs, B):
    """Hub rows (1500-2900 nonzeros) go through the long-row kernel in every launch shape."""
    n, K, t = 6000, 7, 1.5
    arrs = synth.random_local_graph(n, 6, 300, np.random.default_rng(21), hubs=4, hub_degree=2900)
    assert np.diff(arrs[0]).max() > 1500
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    x = synth.random_dense_like(n, B, np.random.default_rng(22))
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    for flags in (0, gs.GS_PLAN_NO_GRAPH):
        plan = gs.Plan(g, K, B, flags=flags)
        Y = torch.empty(n * B, device="cuda")
        for shape in _shapes(B):
            plan.set_shape(*shape)
            plan.set_csr_hint(shape[1] % 2 == 0)   # hub rows through both CSR load forms
            gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
            err = np.abs(to_host(Y).reshape(n, B) - ref).max()
            assert err <= heat_tol(K, np.abs(x).max()), (shape, err)


def test_heat_apply_time_derivative(gs, swiss):
    X, arrs, L, info, A = swiss
    n, K, t, B = 2000, 30, 2.0, 8
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = synth.random_dense_like(n, B, np.random.default_rng(5))
    plan = gs.Plan(g, K, B)
    Y = torch.empty(n * B, device="cuda")
    Yd = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y, Yd)
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    refd = heat.heat_apply_dt(L, lam, t, K, x.astype(np.float64))
    tol = heat_tol(K, np.abs(x).max())
    assert np.abs(to_host(Y).reshape(n, B) - ref).max() <= tol
    assert np.abs(to_host(Yd).reshape(n, B) - refd).max() <= 2 * tol


def test_autotuned_plan_agrees(gs, swiss, tmp_path):
    X, arrs, L, info, A = swiss
    n, K, t, B = 2000, 20, 1.0, 32
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    x = synth.random_dense_like(n, B, np.random.default_rng(9))
    cache = str(tmp_path / "tune.json")
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=cache)
    assert "autotuned" in plan.describe()
    again = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=cache)
    assert "cache" in again.describe()
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    assert np.abs(to_host(Y).reshape(n, B) - ref).max() <= heat_tol(K, np.abs(x).max())


def test_graph_replay_is_bitwise_equal_to_direct_launches(gs, swiss):
    X, arrs, L, info, A = swiss
    n, K, t, B = 2000, 20, 1.0, 16
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    xd = to_dev(synth.random_dense_like(n, B, np.random.default_rng(11)))
    outs = []
    for flags in (0, gs.GS_PLAN_NO_GRAPH):
        plan = gs.Plan(g, K, B, flags=flags)
        Y = torch.empty(n * B, device="cuda")
        for _ in range(3):  # replays with eager work in between
            gs.gs_heat_apply(plan, lam, t, xd, Y)
            torch.cuda.synchronize()
            outs.append(Y.clone())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("B", [1, 4])
def test_cycle_one_million_nodes_closed_form(gs, B):
    n, K, t, lam = 1_000_000, 50, 2.0, 4.0
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    x = synth.random_dense_like(n, B, np.random.default_rng(B))
    plan = gs.Plan(g, K, B)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = closed_forms.cycle_heat_apply(n, lam, t, K, x.astype(np.float64))
    assert np.abs(to_host(Y).reshape(n, B) - ref).max() <= heat_tol(K, np.abs(x).max())


def test_knn_sized_random_graph_one_million_nodes(gs):
    """n = 1M, ~15M nonzeros, B = 32 with K = 50: the batched workload's operator size."""
    n, K, t, B = 1_000_000, 50, 2.0, 32
    arrs = synth.random_local_graph(n, 8, 20000, np.random.default_rng(5))
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    x = synth.random_dense_like(n, B, np.random.default_rng(6))
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    cols = [0, 13, 31]
    ref = heat.heat_apply(L, lam, t, K, x[:, cols].astype(np.float64))
    err = np.abs(to_host(Y).reshape(n, B)[:, cols] - ref).max()
    assert err <= heat_tol(K, np.abs(x).max()), (err, plan.describe())

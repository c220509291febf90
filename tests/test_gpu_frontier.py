"""Frontier-sparse steps (gs_plan_set_frontier): the dense results, bit for bit.

T_k(y) x vanishes beyond k hops of supp(x) (Sec. "Chebyshev Polynomials": y
couples a node only to itself and its neighbours), so step k may skip the rows
more than k hops from the applied support.  Every case runs the same plan with
the option off and on and compares the outputs bit for bit (int32 views, so
signs of zeros count too), and compares them with the float64 oracle: heat
applications from localised supports (single nodes on a path and a cycle,
a few nodes on a banded graph with hub rows; K = 1..4, 20, 256; B = 1, 3, 32;
both polynomial kernels; every launch shape; the time derivative; two calls
with different supports on one plan; all-zero and full supports, a graph
smaller than one row block), Algorithm 1 with and without vertex weights
(some of them zero), with checkpoints and with records and the reverse sweep
from them, iteration counts 1, 2, 5, 1, 3 on one plan, a barycenter on a plan
whose Sinkhorn calls ran with the option, and the backward-Euler kernel,
which ignores it.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph  # noqa: F401
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


def bits(t):
    return t.detach().contiguous().view(torch.int32).cpu()


def same_bits(a, b):
    return torch.equal(bits(a), bits(b))


@pytest.fixture(scope="module")
def graphs():
    """6000 nodes, 3 partners within 20 ids: a band whose k-hop neighbourhoods
    grow by about 40 nodes a hop; and the same with 4 hub rows of 2900 random
    partners (the long-row blocks), which reach most rows within 3 hops."""
    n = 6000
    out = {}
    for name, hubs in (("band", 0), ("hubs", 4)):
        arrs = synth.random_local_graph(n, 3, 20, np.random.default_rng(31), hubs=hubs, hub_degree=2900)
        out[name] = (n, arrs, csr_laplacian(n, arrs))
    return out


@pytest.fixture(scope="module")
def hubgraph(graphs):
    return graphs["hubs"]


def local_columns(n, B, rng, nodes_per_col=3):
    """n x B histograms, each column on a few random nodes."""
    X = np.zeros((n, B), dtype=np.float32)
    for c in range(B):
        X[rng.choice(n, nodes_per_col, replace=False), c] = rng.uniform(0.5, 2.0, nodes_per_col)
    return X


def apply_both(gs, plan, lam, t, X, dt=False):
    n, B = X.shape
    out = {}
    for fr in (0, 1):
        plan.set_frontier(fr)
        Y = torch.full((n * B,), np.nan, device="cuda")
        Yd = torch.full((n * B,), np.nan, device="cuda") if dt else None
        gs.gs_heat_apply(plan, lam, t, to_dev(X), Y, Yd)
        out[fr] = (Y, Yd)
    assert "frontier=on" in plan.describe()
    return out


@pytest.mark.parametrize("graph", ["band", "hubs"])
@pytest.mark.parametrize("kernel", ["chebyshev", "clenshaw"])
@pytest.mark.parametrize("B", [1, 3, 32])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 20])
def test_frontier_heat_apply_bitwise(gs, graphs, graph, kernel, B, K):
    n, arrs, L = graphs[graph]
    t = 1.0
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    X = local_columns(n, B, np.random.default_rng(100 * K + B))
    plan = gs.Plan(g, K, B)
    if kernel == "clenshaw":
        plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
    out = apply_both(gs, plan, lam, t, X)
    assert same_bits(out[0][0], out[1][0]), plan.describe()
    ref = heat.heat_apply(L, lam, t, K, X.astype(np.float64))
    got = to_host(out[1][0]).reshape(n, B)
    assert np.abs(got - ref).max() <= heat_tol(K, np.abs(X).max())
    # rows beyond K hops of every column's support hold exact zeros
    G = sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=(n, n))
    hops = sp.csgraph.shortest_path(G, unweighted=True, indices=np.flatnonzero(X.any(axis=1))).min(axis=0)
    if graph == "band" and K * B <= 64:
        assert np.count_nonzero(hops > K) > 0
    assert np.all(got[hops > K] == 0.0)


@pytest.mark.parametrize("graph", ["band", "hubs"])
@pytest.mark.parametrize("B", [1, 10])
def test_frontier_every_launch_shape(gs, graphs, graph, B):
    """Every launch shape, direct launches and captured graphs, both kernels."""
    n, arrs, L = graphs[graph]
    K, t = 9, 1.5
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    X = local_columns(n, B, np.random.default_rng(7 + B), nodes_per_col=2)
    ref = heat.heat_apply(L, lam, t, K, X.astype(np.float64))
    if B == 1:
        shapes = [(1, S, 1) for S in (2, 4, 8, 16, 32, 64)]
    else:
        ldp = (B + 3) // 4 * 4
        shapes = [(4, S, C) for C in (1, 2, 4, 8, 16, 32, 64) if C == 1 or C // 2 < ldp // 4
                  for S in (1, 2, 4, 8, 16) if S * C <= 64]
    for flags in (0, gs.GS_PLAN_NO_GRAPH):
        for kernel in (gs.GS_KERNEL_CHEBYSHEV, gs.GS_KERNEL_CLENSHAW):
            plan = gs.Plan(g, K, B, flags=flags)
            for shape in shapes:
                plan.set_shape(*shape)
                plan.set_kernel(kernel)
                out = apply_both(gs, plan, lam, t, X)
                assert same_bits(out[0][0], out[1][0]), (shape, plan.describe())
                err = np.abs(to_host(out[1][0]).reshape(n, B) - ref).max()
                assert err <= heat_tol(K, np.abs(X).max()), (shape, err)


def test_frontier_time_derivative(gs, hubgraph):
    n, arrs, L = hubgraph
    K, t, B = 12, 2.0, 8
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    X = local_columns(n, B, np.random.default_rng(5))
    plan = gs.Plan(g, K, B)
    out = apply_both(gs, plan, lam, t, X, dt=True)
    assert same_bits(out[0][0], out[1][0]) and same_bits(out[0][1], out[1][1])
    tol = heat_tol(K, np.abs(X).max())
    assert np.abs(to_host(out[1][1]).reshape(n, B) - heat.heat_apply_dt(L, lam, t, K, X.astype(np.float64))).max() \
        <= 2 * tol


def test_frontier_two_calls_move_the_support(gs, hubgraph):
    """The levels follow each call's X (recomputed inside the replayed graph)."""
    n, arrs, L = hubgraph
    K, t, B = 6, 1.0, 4
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    dense = gs.Plan(g, K, B)
    plan = gs.Plan(g, K, B)
    plan.set_frontier(1)
    for seed in (1, 2, 3):
        X = local_columns(n, B, np.random.default_rng(seed))
        Y0 = torch.empty(n * B, device="cuda")
        Y1 = torch.empty(n * B, device="cuda")
        gs.gs_heat_apply(dense, lam, t, to_dev(X), Y0)
        gs.gs_heat_apply(plan, lam, t, to_dev(X), Y1)
        assert same_bits(Y0, Y1), seed


@pytest.mark.parametrize("kernel", ["chebyshev", "clenshaw"])
@pytest.mark.parametrize("K", [50, 256])
def test_frontier_cycle_single_node(gs, K, kernel):
    """One node on a cycle: the frontier grows one hop per step, so almost
    every block leaves at once on every step but the last; K = 256 (the
    largest degree) on a 2000-node cycle, where the frontier covers half the
    rows by the last step."""
    n, t, lam = 100_000 if K == 50 else 2000, 2.0, 4.0
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    X = np.zeros((n, 1), dtype=np.float32)
    X[n // 3, 0] = 1.0
    plan = gs.Plan(g, K, 1)
    if kernel == "clenshaw":
        plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
    out = apply_both(gs, plan, lam, t, X)
    assert same_bits(out[0][0], out[1][0])
    ref = closed_forms.cycle_heat_apply(n, lam, t, K, X.astype(np.float64))
    got = to_host(out[1][0]).reshape(n, 1)
    assert np.abs(got - ref).max() <= heat_tol(K, 1.0)
    d = np.abs(np.arange(n) - n // 3)
    d = np.minimum(d, n - d)
    assert np.all(got[d > K] == 0.0) and np.all(got[d <= min(K, 20)] != 0.0)


def sinkhorn_both(gs, plan, lam, t, mu, nu, J, a=None, ce=0):
    n, B = mu.shape
    res = {}
    for fr in (0, 1):
        plan.set_frontier(fr)
        v = torch.full((n * B,), np.nan, device="cuda")
        w = torch.full((n * B,), np.nan, device="cuda")
        ck = torch.zeros(gs.ckpt_floats(plan, J, ce), device="cuda") if ce else None
        out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, a=None if a is None else to_dev(a),
                             ckpt_every=ce, ckpt=ck, v=v, w=w, want_marg=True, want_floors=True)
        res[fr] = (out, v, w, ck)
    o0, o1 = res[0][0], res[1][0]
    assert np.array_equal(o0["dist"].view(np.int64), o1["dist"].view(np.int64))
    assert np.array_equal(o0["marg_err"].view(np.int64), o1["marg_err"].view(np.int64))
    assert o0["n_floored"] == o1["n_floored"]
    for i in (1, 2, 3):
        if res[0][i] is not None:
            assert same_bits(res[0][i], res[1][i]), i
    return res


@pytest.fixture(scope="module")
def curve():
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    return X.shape[0], labels, arrs, L


@pytest.mark.parametrize("kernel", ["chebyshev", "clenshaw"])
@pytest.mark.parametrize("weights", [False, True])
def test_frontier_sinkhorn_bitwise(gs, curve, kernel, weights):
    """Localised pairs (two neighbouring clusters each) on the 3000-node curve."""
    n, labels, arrs, L = curve
    K, t, J, B = 10, 1.0, 30, 4
    rng = np.random.default_rng(8)
    pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in (0, 2, 4, 6)]
    mu = np.stack([p[0] for p in pairs], axis=1).astype(np.float32)
    nu = np.stack([p[1] for p in pairs], axis=1).astype(np.float32)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32) if weights else None
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    if kernel == "clenshaw":
        plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
    res = sinkhorn_both(gs, plan, lam, t, mu, nu, J, a=a)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J,
                       a=None if a is None else a.astype(np.float64))
    out = res[1][0]
    assert out["n_floored"] == ref["n_floored"]
    assert np.all(np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t))


@pytest.mark.parametrize("ce", [5, -1])
def test_frontier_checkpoints_records_and_reverse_sweep(gs, curve, ce):
    """The checkpoints or records a frontier forward writes are the dense ones;
    the reverse sweep from them gives the oracle's gradients."""
    n, labels, arrs, L = curve
    K, t, J, B = 15, 2.0, 12, 4
    rng = np.random.default_rng(8)
    pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in (0, 2, 4, 6)]
    mu = np.stack([p[0] for p in pairs], axis=1).astype(np.float32)
    nu = np.stack([p[1] for p in pairs], axis=1).astype(np.float32)
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    ce = gs.GS_RECORD_ALL if ce < 0 else ce
    res = sinkhorn_both(gs, plan, lam, t, mu, nu, J, ce=ce)
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, to_dev(mu), to_dev(nu), J, ce, res[1][3], np.ones(B),
                                 grad_mu=gmu, grad_nu=gnu)
    for got, want, h in ((gmu, ref["dmu"], mu), (gnu, ref["dnu"], nu)):
        G = to_host(got).reshape(n, B)
        s = h > 0
        assert np.linalg.norm(G[s] - want[s]) / np.linalg.norm(want[s]) <= 1e-4
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)


def test_frontier_sinkhorn_far_pairs_floor_alike(gs):
    """Supports more than K hops apart on a cycle: p_K(a w) is exactly zero on
    supp(mu), every denominator of the first scaling floors, in both forms."""
    n, K, t, J = 20_000, 8, 1.0, 3
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    mu = np.zeros((n, 1), dtype=np.float32)
    nu = np.zeros((n, 1), dtype=np.float32)
    mu[100:110, 0] = 0.1
    nu[5000:5010, 0] = 0.1
    plan = gs.Plan(g, K, 1)
    res = sinkhorn_both(gs, plan, 4.0, t, mu, nu, J)
    assert res[1][0]["n_floored"] > 0


def test_frontier_second_sinkhorn_call_and_barycenter(gs, curve):
    """New pairs on the same plan recompute the levels; a barycenter on a plan
    whose Sinkhorn calls ran with the option keeps its own dense graphs."""
    n, labels, arrs, L = curve
    K, t, J, B = 10, 1.0, 20, 4
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    dense = gs.Plan(g, K, B)
    plan.set_frontier(1)
    for seed, starts in ((8, (0, 2, 4, 6)), (9, (1, 3, 5, 7))):
        rng = np.random.default_rng(seed)
        pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in starts]
        mu = to_dev(np.stack([p[0] for p in pairs], axis=1))
        nu = to_dev(np.stack([p[1] for p in pairs], axis=1))
        o = [gs.gs_sinkhorn(p, lam, t, mu, nu, J, want_marg=True) for p in (dense, plan)]
        assert np.array_equal(o[0]["dist"], o[1]["dist"]) and np.array_equal(o[0]["marg_err"], o[1]["marg_err"])
    H, _ = synth.loguniform_support_histograms(n, B, 30, 1500, 0.5, np.random.default_rng(3))
    alpha = np.full(B, 1.0 / B)
    bary = [torch.empty(n, device="cuda") for _ in range(2)]
    outs = [gs.gs_barycenter(p, lam, t, to_dev(H), alpha, 15, bb, want_marg=True)
            for p, bb in ((dense, bary[0]), (plan, bary[1]))]
    assert same_bits(bary[0], bary[1])
    assert np.array_equal(outs[0]["marg_err"], outs[1]["marg_err"])


def test_frontier_sinkhorn_iteration_counts_share_a_plan(gs, curve):
    """J = 1, 2, 5, 1, 3 on one plan: the first application from each support
    advances its levels (at J = 1 that is the marginal check's), the captured
    graphs of one count never serve another wrongly."""
    n, labels, arrs, L = curve
    K, t, B = 10, 1.0, 4
    lam = lam_hat_of(L)
    rng = np.random.default_rng(12)
    pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in (0, 2, 4, 6)]
    mu = to_dev(np.stack([p[0] for p in pairs], axis=1))
    nu = to_dev(np.stack([p[1] for p in pairs], axis=1))
    g = gs.gs_graph_from_csr(n, *arrs)
    dense = gs.Plan(g, K, B)
    plan = gs.Plan(g, K, B)
    plan.set_frontier(1)
    for J in (1, 2, 5, 1, 3):
        vw = [[torch.empty(n * B, device="cuda") for _ in range(2)] for _ in range(2)]
        o = [gs.gs_sinkhorn(p, lam, t, mu, nu, J, v=x[0], w=x[1], want_marg=True)
             for p, x in ((dense, vw[0]), (plan, vw[1]))]
        assert np.array_equal(o[0]["dist"], o[1]["dist"]), J
        assert np.array_equal(o[0]["marg_err"], o[1]["marg_err"]), J
        assert same_bits(vw[0][0], vw[1][0]) and same_bits(vw[0][1], vw[1][1]), J


def test_frontier_degenerate_supports(gs, graphs):
    """An all-zero X (every row beyond every step: the result is exactly zero),
    an all-zero column beside a one-node one, a single row block's worth of
    graph (n below the rows of one block) and a support covering every row."""
    n, arrs, L = graphs["band"]
    K, t = 7, 1.0
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    plan = gs.Plan(g, K, 4)
    X = np.zeros((n, 4), dtype=np.float32)
    out = apply_both(gs, plan, lam, t, X)
    assert same_bits(out[0][0], out[1][0]) and np.all(to_host(out[1][0]) == 0.0)
    X[123, 1] = 1.0
    out = apply_both(gs, plan, lam, t, X)
    assert same_bits(out[0][0], out[1][0])
    X[:] = np.random.default_rng(4).uniform(0.1, 1.0, X.shape)
    out = apply_both(gs, plan, lam, t, X)
    assert same_bits(out[0][0], out[1][0])

    m = 10   # fewer rows than one block of any launch shape
    gsm = gs.gs_graph_from_csr(m, *synth.cycle_graph(m))
    small = gs.Plan(gsm, 3, 1)
    x = np.zeros((m, 1), dtype=np.float32)
    x[2, 0] = 1.0
    out = apply_both(gs, small, 4.0, t, x)
    assert same_bits(out[0][0], out[1][0])
    ref = closed_forms.cycle_heat_apply(m, 4.0, t, 3, x.astype(np.float64))
    assert np.abs(to_host(out[1][0]).reshape(m, 1) - ref).max() <= heat_tol(3, 1.0)


def test_frontier_with_zero_vertex_weights(gs, curve):
    """Vertex weights that vanish on part of the supports shrink supp(a w)
    below supp(nu): the levels from supp(nu) stay a valid (looser) bound."""
    n, labels, arrs, L = curve
    K, t, J, B = 10, 1.0, 15, 4
    rng = np.random.default_rng(21)
    pairs = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in (0, 2, 4, 6)]
    mu = np.stack([p[0] for p in pairs], axis=1).astype(np.float32)
    nu = np.stack([p[1] for p in pairs], axis=1).astype(np.float32)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    a[rng.choice(n, n // 3, replace=False)] = 0.0
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    sinkhorn_both(gs, plan, lam, t, mu, nu, J, a=a)


def test_frontier_option_leaves_the_euler_kernel_alone(gs, graphs):
    """The backward-Euler kernel ignores the option: the same results with it on."""
    n, arrs, L = graphs["band"]
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    X = local_columns(n, 4, np.random.default_rng(2))
    plan = gs.Plan(g, 12, 4)
    plan.set_kernel(gs.GS_KERNEL_EULER, 4, 0)
    out = apply_both(gs, plan, lam, 0.5, X)
    assert same_bits(out[0][0], out[1][0])
    assert "kernel=euler" in plan.describe()


def test_frontier_setter_rejects_other_values(gs, graphs):
    from paper_2211_00805_amd import _lib
    n, arrs, L = graphs["band"]
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, 5, 1)
    for bad in (2, -1):
        with pytest.raises(gs.GeoSinkError, match="enable must be 0 or 1"):
            _lib.check("gs_plan_set_frontier", _lib.lib.gs_plan_set_frontier(plan.handle, bad))
    assert "frontier=on" not in plan.describe()
    plan.set_frontier(True)
    assert "frontier=on" in plan.describe()
    plan.set_frontier(False)
    assert "frontier=on" not in plan.describe()

"""Pins for the oracle's Algorithm 1, barycenter and reverse-mode gradient.

Independent routes: exact two-node values (golden), one-dimensional convex
minimisation over 2x2 couplings, the entropic dual solved by L-BFGS,
primal = dual at the fixed point, symmetry in (mu, nu), the m = 1 barycenter
closed form, a nested search for the two-node barycenter, and central finite
differences for the gradient.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import closed_forms, graph, heat, sinkhorn, spectrum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def edge_laplacian(w=1.0):
    A = graph.csr_from_arrays(2, [0, 1, 2], [1, 0], [w, w])
    return graph.laplacian(A)


def tiny_graph(n=10, k=4, seed=0):
    X = np.random.default_rng(seed).standard_normal((n, 3))
    A, info = graph.knn_graph(X, k)
    assert info["n_components"] == 1
    L = graph.laplacian(A)
    return L, 1.01 * spectrum.lambda_max(L)


def rand_hist(n, rng, support=None):
    h = np.zeros(n)
    s = np.arange(n) if support is None else support
    h[s] = rng.uniform(0.2, 1.0, size=len(s))
    return h / h.sum()


@pytest.mark.parametrize("t", [0.5, 1.0, 2.0])
def test_two_node_dirac_golden(t):
    with open(os.path.join(GOLDEN, "two_node.json")) as f:
        ref = json.load(f)["D_exact"][str(t)]
    L = edge_laplacian()
    out = sinkhorn.sinkhorn(L, 2.0, t, 60, np.array([1.0, 0.0]), np.array([0.0, 1.0]), 3)
    assert out["D"][0] == pytest.approx(ref, rel=1e-12)
    # low order: equals the closed form with the polynomial's own H_12
    out5 = sinkhorn.sinkhorn(L, 2.0, t, 5, np.array([1.0, 0.0]), np.array([0.0, 1.0]), 3)
    assert out5["D"][0] == pytest.approx(closed_forms.two_node_dirac_distance(t, 5), rel=1e-13)


@pytest.mark.parametrize("t", [0.3, 1.0])
def test_two_node_general_matches_coupling_search(t):
    L = edge_laplacian()
    mu, nu = np.array([0.3, 0.7]), np.array([0.6, 0.4])
    out = sinkhorn.sinkhorn(L, 2.0, t, 40, mu, nu, 400)
    ref = closed_forms.two_node_plan_cost(closed_forms.two_node_kernel(t, 40), mu, nu)
    assert out["D"][0] / (4 * t) == pytest.approx(ref, rel=1e-9, abs=1e-12)


def test_matches_entropic_dual_solved_by_lbfgs():
    L, lam = tiny_graph(n=9, k=4, seed=2)
    t, K = 1.0, 30
    rng = np.random.default_rng(0)
    mu, nu = rand_hist(9, rng, [0, 2, 3, 5]), rand_hist(9, rng, [1, 4, 6, 7, 8])
    out = sinkhorn.sinkhorn(L, lam, t, K, mu, nu, 3000)
    P = heat.heat_dense_poly(L, lam, t, K)
    ref = closed_forms.dual_ascent_distance(P, mu, nu)
    assert out["D"][0] / (4 * t) == pytest.approx(ref, rel=1e-7)


def test_fixed_point_identities():
    L, lam = tiny_graph(n=12, k=4, seed=4)
    n = 12
    t, K = 1.3, 25
    rng = np.random.default_rng(1)
    mu, nu = rand_hist(n, rng), rand_hist(n, rng)
    out = sinkhorn.sinkhorn(L, lam, t, K, mu, nu, 3000)
    assert out["marg_row"][0] < 1e-12 and out["marg_col"][0] < 1e-12
    P = heat.heat_dense_poly(L, lam, t, K)
    pi = out["v"][:, None] * P * out["w"][None, :]
    np.testing.assert_allclose(pi.sum(axis=1), mu, atol=1e-12)
    primal = 4 * t * np.sum(pi * np.log(pi / P))
    assert out["D"][0] == pytest.approx(primal, rel=1e-10)
    swapped = sinkhorn.sinkhorn(L, lam, t, K, nu, mu, 3000)
    assert swapped["D"][0] == pytest.approx(out["D"][0], rel=1e-10)
    p0 = 0.5 * heat.cheb_coeffs(t, K)[0] + np.sum(heat.cheb_coeffs(t, K)[1:] * (-1.0) ** np.arange(1, K + 1))
    assert out["D"][0] >= -4 * t * np.log(n * p0)


def test_vertex_weights_equal_rescaled_kernel_problem():
    """General a: same as unit-weight OT with kernel diag(a) P diag(a) and marginals a*mu, a*nu."""
    L, lam = tiny_graph(n=8, k=3, seed=6)
    t, K = 0.8, 30
    rng = np.random.default_rng(2)
    a = rng.uniform(0.5, 1.5, size=8)
    mu, nu = rand_hist(8, rng), rand_hist(8, rng)
    mu, nu = mu / np.sum(a * mu), nu / np.sum(a * nu)
    out = sinkhorn.sinkhorn(L, lam, t, K, mu, nu, 3000, a=a)
    P = heat.heat_dense_poly(L, lam, t, K)
    ref = closed_forms.dual_ascent_distance(a[:, None] * P * a[None, :], a * mu, a * nu)
    assert out["D"][0] / (4 * t) == pytest.approx(ref, rel=1e-7)


def _dense_plan(L, lam, t, a, v, w):
    """Explicit plan diag(a v) H diag(a w) with H = exp(-t L_op) from a dense
    eigendecomposition (no Chebyshev code; at K = 40, t <= 1 the truncation
    tail is below 1e-40, so p_K equals H to rounding)."""
    H = heat.heat_dense_exact(L, lam, t)
    return (a * v)[:, None] * H * (a * w)[None, :]


def test_row_marginal_with_vertex_weights_equals_dense_plan_row_sums():
    """The plan comparator: a v p_K(a w) is the row sum of the explicit plan
    diag(a v) H diag(a w) (Algorithm 1's plan with vertex weights a; Sec.
    "Sinkhorn Distances": plan diag(v) K diag(w)), for arbitrary positive
    scalings v, w (not only at a fixed point) and several columns.  Dropping
    a from either side, or applying it once, fails."""
    L, lam = tiny_graph(n=11, k=4, seed=12)
    t, K = 0.9, 40
    rng = np.random.default_rng(31)
    a = rng.uniform(0.3, 2.0, size=11)
    V = rng.uniform(0.1, 3.0, size=(11, 3))
    W = rng.uniform(0.1, 3.0, size=(11, 3))
    got = sinkhorn.row_marginal(L, lam, t, K, V, W, a=a)
    for c in range(3):
        ref = _dense_plan(L, lam, t, a, V[:, c], W[:, c]).sum(axis=1)
        np.testing.assert_allclose(got[:, c], ref, rtol=1e-12, atol=1e-15)
    # a = None means unit weights
    ref1 = _dense_plan(L, lam, t, np.ones(11), V[:, 0], W[:, 0]).sum(axis=1)
    np.testing.assert_allclose(sinkhorn.row_marginal(L, lam, t, K, V[:, 0], W[:, 0])[:, 0], ref1, rtol=1e-12)


def test_marginal_errors_with_vertex_weights_equal_dense_plan():
    """Algorithm 1's reported marginal violations with vertex weights, after a
    few (unconverged) iterations, equal the L1 distances of the explicit plan's
    row and column sums to a mu and a nu."""
    L, lam = tiny_graph(n=10, k=4, seed=13)
    t, K, J = 0.7, 40, 3
    rng = np.random.default_rng(32)
    a = rng.uniform(0.3, 2.0, size=10)
    mus = np.stack([rand_hist(10, rng, [0, 1, 3, 6, 8]), rand_hist(10, rng)], axis=1)
    nus = np.stack([rand_hist(10, rng, [2, 4, 5, 7, 9]), rand_hist(10, rng)], axis=1)
    out = sinkhorn.sinkhorn(L, lam, t, K, mus, nus, J, a=a)
    for c in range(2):
        Pi = _dense_plan(L, lam, t, a, out["v"][:, c], out["w"][:, c])
        row = np.abs(Pi.sum(axis=1) - a * mus[:, c]).sum()
        col = np.abs(Pi.sum(axis=0) - a * nus[:, c]).sum()
        assert row > 1e-6                      # unconverged: the pin sees the row side
        assert out["marg_row"][c] == pytest.approx(row, rel=1e-9)
        assert out["marg_col"][c] == pytest.approx(col, rel=1e-6, abs=1e-13)


def test_columns_are_independent_problems():
    L, lam = tiny_graph(n=10, k=4, seed=8)
    rng = np.random.default_rng(3)
    mus = np.stack([rand_hist(10, rng) for _ in range(3)], axis=1)
    nus = np.stack([rand_hist(10, rng) for _ in range(3)], axis=1)
    both = sinkhorn.sinkhorn(L, lam, 1.0, 20, mus, nus, 50)
    for c in range(3):
        one = sinkhorn.sinkhorn(L, lam, 1.0, 20, mus[:, c], nus[:, c], 50)
        assert both["D"][c] == pytest.approx(one["D"][0], rel=1e-14)


def test_floors_are_counted_beyond_receptive_field():
    n = 40
    path = graph.csr_from_arrays(n, *synth.cycle_graph(n))   # cycle: far side is > K hops away
    L = graph.laplacian(path)
    mu = np.zeros(n); mu[0] = 1.0
    nu = np.zeros(n); nu[20] = 1.0
    out = sinkhorn.sinkhorn(L, 4.0, 1.0, 5, mu, nu, 2)
    assert out["n_floored"] > 0
    ok = sinkhorn.sinkhorn(L, 4.0, 1.0, 25, mu, nu, 2)
    assert ok["n_floored"] == 0


# ---------------------------------------------------------------- barycenter

def test_barycenter_single_input_closed_form():
    L, lam = tiny_graph(n=14, k=4, seed=10)
    t, K = 1.0, 25
    rng = np.random.default_rng(4)
    mu = rand_hist(14, rng, [1, 3, 4, 9])
    out = sinkhorn.barycenter(L, lam, t, K, mu[:, None], np.array([1.0]), 5)
    b = heat.cheb_coeffs(t, K)
    p0 = 0.5 * b[0] + np.sum(b[1:] * (-1.0) ** np.arange(1, K + 1))
    np.testing.assert_allclose(out["p"], heat.heat_apply(L, lam, t, K, mu) / p0, atol=1e-14)


def test_two_node_barycenter_matches_nested_search():
    L = edge_laplacian()
    t, K = 0.7, 40
    mus = np.array([[0.9, 0.2], [0.1, 0.8]])
    alpha = np.array([0.3, 0.7])
    out = sinkhorn.barycenter(L, 2.0, t, K, mus, alpha, 2000)
    ref = closed_forms.two_node_barycenter(closed_forms.two_node_kernel(t, K), mus, alpha)
    np.testing.assert_allclose(out["p"], ref, atol=2e-6)
    assert abs(out["p"].sum() - 1.0) < 1e-10


def test_barycenter_input_permutation_and_duplicates():
    L, lam = tiny_graph(n=12, k=4, seed=12)
    rng = np.random.default_rng(5)
    mus = np.stack([rand_hist(12, rng) for _ in range(3)], axis=1)
    alpha = np.array([0.2, 0.5, 0.3])
    a = sinkhorn.barycenter(L, lam, 1.0, 20, mus, alpha, 200)
    perm = [2, 0, 1]
    b = sinkhorn.barycenter(L, lam, 1.0, 20, mus[:, perm], alpha[perm], 200)
    np.testing.assert_allclose(a["p"], b["p"], atol=1e-14)
    one = sinkhorn.barycenter(L, lam, 1.0, 20, mus[:, :1], np.array([1.0]), 50)
    dup = sinkhorn.barycenter(L, lam, 1.0, 20, np.repeat(mus[:, :1], 3, axis=1), alpha, 50)
    np.testing.assert_allclose(dup["p"], one["p"], atol=1e-14)
    assert a["marg_row"].max() < 1e-8


# ---------------------------------------------------------------- gradient

def test_gradient_matches_finite_differences():
    L, lam = tiny_graph(n=12, k=4, seed=14)
    t, K, J = 1.3, 25, 30
    rng = np.random.default_rng(6)
    mu = rand_hist(12, rng, [0, 1, 4, 5, 7, 9])
    nu = rand_hist(12, rng, [2, 3, 6, 8, 10, 11, 4])
    g = sinkhorn.sinkhorn_grad(L, lam, t, K, mu, nu, J)
    coords = np.nonzero(mu > 0)[0]
    fd = sinkhorn.finite_diff_mu(L, lam, t, K, mu, nu, J, coords)
    np.testing.assert_allclose(g["dmu"][coords], fd, rtol=1e-6)
    fdn = sinkhorn.finite_diff_mu(L, lam, t, K, nu, mu, J, np.nonzero(nu > 0)[0])
    gs = sinkhorn.sinkhorn_grad(L, lam, t, K, nu, mu, J)
    np.testing.assert_allclose(gs["dmu"][nu > 0], fdn, rtol=1e-6)
    fdt = sinkhorn.finite_diff_t(L, lam, t, K, mu, nu, J)
    assert g["dt"][0] == pytest.approx(fdt[0], rel=1e-6)


def test_gradient_with_vertex_weights_and_column_weights():
    L, lam = tiny_graph(n=10, k=4, seed=16)
    t, K, J = 0.9, 20, 15
    rng = np.random.default_rng(7)
    a = rng.uniform(0.5, 1.5, size=10)
    mus = np.stack([rand_hist(10, rng, [0, 2, 5, 7]), rand_hist(10, rng, [1, 3])], axis=1)
    nus = np.stack([rand_hist(10, rng, [4, 6, 8]), rand_hist(10, rng, [5, 9, 0])], axis=1)
    gw = np.array([0.7, -1.3])
    g = sinkhorn.sinkhorn_grad(L, lam, t, K, mus, nus, J, a=a, g=gw)
    for c in range(2):
        coords = np.nonzero(mus[:, c] > 0)[0]
        fd = sinkhorn.finite_diff_mu(L, lam, t, K, mus[:, c], nus[:, c], J, coords, a=a)
        np.testing.assert_allclose(g["dmu"][coords, c], gw[c] * fd, rtol=1e-6)
        fdt = sinkhorn.finite_diff_t(L, lam, t, K, mus[:, c], nus[:, c], J, a=a)
        assert g["dt"][c] == pytest.approx(gw[c] * fdt[0], rel=1e-6)
        one = sinkhorn.sinkhorn(L, lam, t, K, mus[:, c], nus[:, c], J, a=a, marginals=False)
        assert g["D"][c] == pytest.approx(one["D"][0], rel=1e-14)


def test_gradient_converged_limit_is_4t_log_v_plus_constant():
    L, lam = tiny_graph(n=9, k=4, seed=18)
    t, K, J = 1.0, 20, 400
    rng = np.random.default_rng(8)
    mu, nu = rand_hist(9, rng), rand_hist(9, rng)
    g = sinkhorn.sinkhorn_grad(L, lam, t, K, mu, nu, J)
    v = sinkhorn.sinkhorn(L, lam, t, K, mu, nu, J, marginals=False)["v"]
    resid = g["dmu"] - 4 * t * np.log(v)
    assert np.ptp(resid) < 1e-8 * np.abs(g["dmu"]).max()

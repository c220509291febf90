"""Pins for the oracle's heat-kernel application p_K(L, t) x.

Checked against: dense eigendecomposition (Sec. "Heat Diffusion on a Graph",
H_t = Psi exp(-t Lambda) Psi^T), scipy's expm_multiply, FFT diagonalisation of
the cycle and the torus, the complete graph's two-point spectrum, and the
invariants symmetry, near-positivity, mass (L 1 = 0) and permutation
equivariance.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

import synth
from oracle import closed_forms, graph, heat, spectrum


def small_knn(n=150, k=6, seed=3):
    X = np.random.default_rng(seed).standard_normal((n, 4))
    A, _ = graph.knn_graph(X, k)
    return A, graph.laplacian(A)


def csr(arrs, n):
    return graph.csr_from_arrays(n, *arrs)


@pytest.mark.parametrize("t,K", [(0.5, 10), (1.0, 20), (2.0, 30), (8.0, 30)])
def test_apply_matches_eigendecomposition(t, K):
    A, L = small_knn()
    lam = 1.01 * spectrum.lambda_max(L)
    x = np.random.default_rng(0).standard_normal((L.shape[0], 3))
    exact = heat.heat_dense_exact(L, lam, t) @ x
    got = heat.heat_apply(L, lam, t, K, x)
    tail = heat.tail_bound(t, K)
    assert np.linalg.norm(got - exact, axis=0).max() <= tail * np.linalg.norm(x, axis=0).max() + 1e-12


def test_apply_matches_expm_multiply():
    A, L = small_knn(n=200, k=8, seed=5)
    lam = 1.05 * spectrum.lambda_max(L)
    t, K = 2.0, 40
    x = np.random.default_rng(1).standard_normal(L.shape[0])
    ref = expm_multiply(-t * (2.0 / lam) * L, x)
    np.testing.assert_allclose(heat.heat_apply(L, lam, t, K, x), ref, atol=1e-12)


@pytest.mark.parametrize("n", [64, 257])
def test_cycle_fft_closed_form(n):
    L = graph.laplacian(csr(synth.cycle_graph(n), n))
    t, K, lam = 2.0, 30, 4.0
    x = np.random.default_rng(n).standard_normal((n, 2))
    np.testing.assert_allclose(heat.heat_apply(L, lam, t, K, x),
                               closed_forms.cycle_heat_apply(n, lam, t, K, x), atol=1e-13)


def test_torus_fft_closed_form():
    n1, n2 = 8, 13
    n = n1 * n2
    L = graph.laplacian(csr(synth.torus_graph(n1, n2), n))
    t, K, lam = 1.0, 25, 8.0
    x = np.random.default_rng(2).standard_normal(n)
    np.testing.assert_allclose(heat.heat_apply(L, lam, t, K, x),
                               closed_forms.torus_heat_apply(n1, n2, lam, t, K, x), atol=1e-13)


def test_complete_graph_closed_form():
    n = 30
    L = graph.laplacian(csr(synth.complete_graph(n), n))
    t, K = 1.3, 25
    x = np.random.default_rng(3).standard_normal((n, 2))
    np.testing.assert_allclose(heat.heat_apply(L, float(n), t, K, x),
                               closed_forms.complete_heat_apply(n, t, K, x), atol=1e-13)
    # limit form: e^{-2t} x + (1 - e^{-2t}) mean(x)
    lim = np.exp(-2 * t) * x + (1 - np.exp(-2 * t)) * x.mean(axis=0, keepdims=True)
    np.testing.assert_allclose(heat.heat_apply(L, float(n), t, K, x), lim, atol=1e-12)


def test_symmetry_positivity_mass_permutation():
    A, L = small_knn(n=120, k=5, seed=9)
    n = L.shape[0]
    lam = 1.01 * spectrum.lambda_max(L)
    t, K = 2.0, 30
    P = heat.heat_dense_poly(L, lam, t, K)
    assert np.abs(P - P.T).max() < 1e-13
    assert P.min() >= -heat.tail_bound(t, K) - 1e-14
    b = heat.cheb_coeffs(t, K)
    p0 = 0.5 * b[0] + np.sum(b[1:] * (-1.0) ** np.arange(1, K + 1))
    x = np.random.default_rng(4).standard_normal(n)
    assert abs(np.sum(heat.heat_apply(L, lam, t, K, x)) - p0 * np.sum(x)) < 1e-12
    perm = np.random.default_rng(5).permutation(n)
    Pm = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))
    Lp = (Pm @ L @ Pm.T).tocsr()
    np.testing.assert_allclose(heat.heat_apply(Lp, lam, t, K, Pm @ x), Pm @ heat.heat_apply(L, lam, t, K, x),
                               atol=1e-13)


def test_time_derivative_matches_finite_difference():
    A, L = small_knn(n=100, k=5, seed=11)
    lam = 1.01 * spectrum.lambda_max(L)
    t, K, h = 2.0, 40, 1e-5
    x = np.random.default_rng(6).standard_normal(L.shape[0])
    fd = (heat.heat_apply(L, lam, t + h, K, x) - heat.heat_apply(L, lam, t - h, K, x)) / (2 * h)
    np.testing.assert_allclose(heat.heat_apply_dt(L, lam, t, K, x), fd, atol=1e-8)


def test_underestimated_lambda_breaks_expansion():
    """lam_hat far below lambda_max maps eigenvalues to y >> 1, where T_k grows
    geometrically; the truncated series then misses the exact kernel by far more
    than the tail bound (which only holds on [-1, 1])."""
    A, L = small_knn(n=150, k=6, seed=13)
    lmax = spectrum.lambda_max(L)
    t, K = 2.0, 30
    x = np.random.default_rng(7).standard_normal(L.shape[0])
    good = heat.heat_apply(L, 1.01 * lmax, t, K, x) - heat.heat_dense_exact(L, 1.01 * lmax, t) @ x
    bad = heat.heat_apply(L, 0.1 * lmax, t, K, x) - heat.heat_dense_exact(L, 0.1 * lmax, t) @ x
    assert np.linalg.norm(good) < 1e-12
    assert np.linalg.norm(bad) > 1e-3


def test_lambda_hat_below_the_spectrum_voids_the_truncation_bound():
    """The rescaling needs lambda_hat >= lambda_max.  Below it, eigenvalues of
    y = (2/lambda_hat) L - I exceed 1, where |T_k(y)| = cosh(k acosh y) > 1:
    the series still expands the entire function exp(-t(y+1)), but the tail
    sum_{k>K} |b_k| no longer bounds the truncation error against
    exp(-t L_op), and once T_K(y_max) outgrows the coefficients' decay the
    truncated sum blows up (no longer a contraction; exp(-t L_op) has
    eigenvalues in (0, 1]).  The mass identity 1^T p_K x = p_K(0) 1^T x holds
    throughout (L 1 = 0 gives y 1 = -1 for every lambda_hat), so it cannot
    reveal a too-small lambda_hat."""
    A, L = small_knn()
    lm = spectrum.lambda_max(L)
    t, K = 8.0, 20
    b = heat.cheb_coeffs(t, K)
    p0 = b[0] / 2 + sum((-1) ** k * b[k] for k in range(1, K + 1))
    tail = heat.tail_bound(t, K)
    x = np.random.default_rng(4).standard_normal(L.shape[0])
    nx = np.linalg.norm(x)
    for ratio, bounded, contraction in ((1.0, True, True), (1.5, True, True), (0.9, False, True),
                                        (0.5, False, False)):
        lam = ratio * lm
        y = heat.heat_apply(L, lam, t, K, x)
        err = np.linalg.norm(y - heat.heat_dense_exact(L, lam, t) @ x)
        assert (err <= tail * nx + 1e-12) == bounded, (ratio, err, tail * nx)
        assert (np.linalg.norm(y) <= (1 + tail) * nx) == contraction, ratio
        assert abs(y.sum() - p0 * x.sum()) <= 1e-9 * max(np.abs(y).sum(), 1.0), ratio


@pytest.mark.parametrize("K", [1, 2, 5, 12])
def test_application_is_local_to_K_hops(K):
    """p_K(L, t) x vanishes exactly beyond K hops of supp(x) and not at K hops.

    y = (2/lambda_hat) L - I couples a node only to itself and its neighbours
    (Sec. "Chebyshev Polynomials"), so T_k(y) x lives on the k-hop
    neighbourhood of supp(x): the fact the frontier-sparse steps rely on.  On a
    path from one end node, the value K hops out is the single walk's weight
    b_K 2^(K-1) (2/lambda_hat)^K prod(-w) (nonzero); every row farther out is
    exactly 0.0.  On a graph with hub rows (and a small diameter), every row
    beyond min(K, 4) hops of a three-node support is exactly 0.0 at that
    degree, and some row at that distance is not.
    """
    n, t = 40, 1.5
    i = np.arange(n - 1)
    w = np.linspace(0.5, 1.5, n - 1)
    A = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([i, i + 1]), np.concatenate([i + 1, i]))),
                      shape=(n, n))
    L = graph.laplacian(A)
    lam = 1.01 * spectrum.lambda_max(L)
    x = np.zeros(n)
    x[0] = 1.0
    y = heat.heat_apply(L, lam, t, K, x)
    assert np.all(y[K + 1:] == 0.0)
    b = heat.cheb_coeffs(t, K)
    walk = b[K] * 2.0 ** (K - 1) * (2.0 / lam) ** K * np.prod(-w[:K])
    assert y[K] == pytest.approx(walk, rel=1e-12) and y[K] != 0.0

    m = 3000
    arrs = synth.random_local_graph(m, 4, 40, np.random.default_rng(K), hubs=2, hub_degree=300)
    G = csr(arrs, m)
    Lg = graph.laplacian(G)
    X = np.zeros((m, 2))
    X[[5, 1700], 0] = [1.0, 2.0]
    X[2900, 1] = 0.5
    hops = sp.csgraph.shortest_path(G, unweighted=True, indices=[5, 1700, 2900]).min(axis=0)
    Kg = min(K, 4)
    Y = heat.heat_apply(Lg, Lg.diagonal().max() * 2.0, t, Kg, X)
    assert np.count_nonzero(hops > Kg) > 100
    assert np.all(Y[hops > Kg] == 0.0)
    assert np.any(Y[hops == Kg] != 0.0)


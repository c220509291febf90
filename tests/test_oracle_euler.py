"""Pins for the oracle's backward-Euler heat kernel (I + (t/N) L_op)^{-N}.

Independent routes: the spectral definition (dense eigendecomposition), the
cycle's Fourier closed form, the residual of one solve, first-order
convergence to exp(-t L_op) as N grows, mass, positivity and symmetry; and
Algorithm 1 with this kernel against the entropic dual optimum of the dense
kernel.  A flipped sign (I - (t/N) L_op), a step of t instead of t/N, or
N - 1 solves each fail the spectral pin.
"""
import numpy as np
import pytest

import synth
from oracle import closed_forms, graph, heat, sinkhorn, spectrum


@pytest.fixture(scope="module")
def small():
    X = np.random.default_rng(3).standard_normal((60, 3))
    A, info = graph.knn_graph(X, 6)
    L = graph.laplacian(A)
    return L, 1.01 * spectrum.lambda_max(L)


@pytest.mark.parametrize("N", [1, 3, 10])
@pytest.mark.parametrize("t", [0.5, 2.0, 8.0])
def test_spectral_definition(small, N, t):
    L, lam = small
    ev, psi = np.linalg.eigh(L.toarray())
    x = np.random.default_rng(N).standard_normal((60, 3))
    ref = psi @ (closed_forms.euler_at_eigs(ev, lam, t, N)[:, None] * (psi.T @ x))
    np.testing.assert_allclose(heat.euler_apply(L, lam, t, N, x), ref, atol=1e-12)


@pytest.mark.parametrize("N", [1, 5, 20])
def test_cycle_closed_form(N):
    n = 2000
    rp, col, w = synth.cycle_graph(n)
    L = graph.laplacian(graph.csr_from_arrays(n, rp, col, w))
    x = np.random.default_rng(7).standard_normal((n, 2))
    np.testing.assert_allclose(heat.euler_apply(L, 4.0, 2.0, N, x), closed_forms.cycle_euler_apply(n, 4.0, 2.0, N, x),
                               atol=1e-12)


def test_one_step_solves_the_system(small):
    L, lam = small
    x = np.random.default_rng(1).standard_normal(60)
    y = heat.euler_apply(L, lam, 1.5, 1, x)
    np.testing.assert_allclose(y + 1.5 * (2.0 / lam) * (L @ y), x, atol=1e-12)


def test_first_order_convergence_to_the_heat_kernel(small):
    L, lam = small
    t = 2.0
    x = np.random.default_rng(2).standard_normal(60)
    exact = heat.heat_dense_exact(L, lam, t) @ x
    errs = [np.abs(heat.euler_apply(L, lam, t, N, x) - exact).max() for N in (50, 100, 200)]
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs


def test_mass_positivity_symmetry(small):
    L, lam = small
    rng = np.random.default_rng(5)
    x, z = rng.uniform(0.1, 1.0, 60), rng.standard_normal(60)
    ex, ez = heat.euler_apply(L, lam, 3.0, 4, x), heat.euler_apply(L, lam, 3.0, 4, z)
    assert abs(ex.sum() - x.sum()) <= 1e-12 * x.sum()
    assert ex.min() > 0
    assert abs(z @ ex - ez @ x) <= 1e-12 * np.linalg.norm(z) * np.linalg.norm(ex)


def test_sinkhorn_with_euler_kernel_reaches_the_dual_optimum(small):
    L, lam = small
    t, N = 1.0, 4
    E = heat.euler_apply(L, lam, t, N, np.eye(60))
    rng = np.random.default_rng(9)
    mu = np.zeros(60)
    nu = np.zeros(60)
    mu[rng.choice(60, 8, replace=False)] = rng.dirichlet(np.ones(8))
    nu[rng.choice(60, 7, replace=False)] = rng.dirichlet(np.ones(7))
    D = sinkhorn.sinkhorn(L, lam, t, 0, mu, nu, 3000, marginals=False,
                          apply=lambda v: heat.euler_apply(L, lam, t, N, v))["D"]
    ref = 4 * t * closed_forms.dual_ascent_distance(E, mu, nu)
    assert D[0] == pytest.approx(ref, rel=1e-7)

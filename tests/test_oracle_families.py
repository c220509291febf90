"""Pins for the oracle's barycentric distance and Expected Barycenter Effect.

Singleton families reduce to the closed-form barycenter p_K mu / p_K(0), so
gamma({mu}, {nu}) must equal Algorithm 1 on those closed forms; the effect is
zero between a family and itself, invariant under shifts of the features,
linear in the features, and for singleton families equals the difference of
the smoothed inputs' feature means.  Against the paper's printed result
(Table 2, Expected Barycenter Effect with one outlier member): on a reduced
copy of that setup (200 samples per member instead of 500) the effect stays
within the paper's reported spread (0.2) of the true shift 5, where the plain
difference of means is near -1.5 or 1.5.  An arithmetic instead of geometric
mean in the barycenter, or an expectation without the division by the mass,
fails it.
"""
import numpy as np
import pytest

from oracle import families, graph, heat, sinkhorn, spectrum


def setup(n=14, seed=0):
    X = np.random.default_rng(seed).standard_normal((n, 2))
    A, info = graph.knn_graph(X, 4)
    assert info["n_components"] == 1
    L = graph.laplacian(A)
    return X, L, 1.01 * spectrum.lambda_max(L)


def hist(n, rng, k):
    h = np.zeros(n)
    h[rng.choice(n, size=k, replace=False)] = rng.uniform(0.2, 1.0, size=k)
    return h / h.sum()


def p0_of(t, K):
    b = heat.cheb_coeffs(t, K)
    return 0.5 * b[0] + np.sum(b[1:] * (-1.0) ** np.arange(1, K + 1))


def test_singleton_families_reduce_to_closed_form():
    X, L, lam = setup()
    t, K = 1.0, 25
    rng = np.random.default_rng(1)
    mu, nu = hist(14, rng, 5), hist(14, rng, 6)
    g, pT, pC = families.barycentric_distance(L, lam, t, K, mu[:, None], [1.0], nu[:, None], [1.0], 5, 200)
    cT = heat.heat_apply(L, lam, t, K, mu) / p0_of(t, K)
    cC = heat.heat_apply(L, lam, t, K, nu) / p0_of(t, K)
    np.testing.assert_allclose(pT, cT, atol=1e-14)
    ref = sinkhorn.sinkhorn(L, lam, t, K, cT, cC, 200, marginals=False)["D"][0]
    assert g == pytest.approx(ref, rel=1e-12)
    tau = families.expected_barycenter_effect(pT, pC, X)
    np.testing.assert_allclose(tau, (cT @ X) / cT.sum() - (cC @ X) / cC.sum(), atol=1e-13)


def test_effect_properties():
    X, L, lam = setup(n=16, seed=2)
    t, K = 0.8, 20
    rng = np.random.default_rng(3)
    fT = np.stack([hist(16, rng, 6) for _ in range(3)], axis=1)
    fC = np.stack([hist(16, rng, 6) for _ in range(4)], axis=1)
    aT, aC = np.full(3, 1 / 3), np.full(4, 1 / 4)
    g, pT, pC = families.barycentric_distance(L, lam, t, K, fT, aT, fC, aC, 100, 100)
    Y = X[:, 0]
    tau = families.expected_barycenter_effect(pT, pC, Y)
    assert families.expected_barycenter_effect(pT, pC, Y + 7.5) == pytest.approx(tau, abs=1e-12)
    assert families.expected_barycenter_effect(pT, pC, 3.0 * Y) == pytest.approx(3.0 * tau, rel=1e-12)
    assert families.expected_barycenter_effect(pT, pT, Y) == pytest.approx(0.0, abs=1e-15)
    # the same family on both sides: the distance is the entropic self-distance of its barycenter
    gs, p1, p2 = families.barycentric_distance(L, lam, t, K, fT, aT, fT, aT, 100, 100)
    ref = sinkhorn.sinkhorn(L, lam, t, K, p1, p1, 100, marginals=False)["D"][0]
    assert gs == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("seed,outlier", [(1, -60.0), (4, -30.0)])
def test_effect_experiment_recovers_the_shift(seed, outlier):
    S = 200
    rng = np.random.default_rng(seed)
    control = [rng.normal(0.0, 1.0, S) for _ in range(10)]
    treat = [rng.normal(5.0, 1.0, S) for _ in range(9)] + [rng.normal(outlier, 1.0, S)]
    pts = np.concatenate(control + treat)[:, None]
    n = pts.shape[0]
    A, info = graph.knn_graph(pts, 10)
    L = graph.laplacian(A)
    lam = 1.01 * spectrum.lambda_max(L)
    fam = np.zeros((n, 20))
    for i in range(20):
        fam[i * S:(i + 1) * S, i] = 1.0 / S
    alpha = np.full(10, 0.1)
    pT = sinkhorn.barycenter(L, lam, 2.0, 30, fam[:, 10:], alpha, 60)["p"]
    pC = sinkhorn.barycenter(L, lam, 2.0, 30, fam[:, :10], alpha, 60)["p"]
    tau = families.expected_barycenter_effect(pT, pC, pts)[0]
    naive = np.mean(np.concatenate(treat)) - np.mean(np.concatenate(control))
    assert abs(tau - 5.0) < 0.2, tau
    assert abs(naive - 5.0) > 3.0

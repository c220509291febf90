"""Pins for the oracle's all-pairs distances and nearest-neighbour scores.

The matrix places Algorithm 1's value for each pair (checked against single
pair runs) symmetrically with a zero diagonal.  Against the paper's printed
result (Table 1, Geodesic Sinkhorn row: Spearman 0.847 +- 0.023, P@5
0.833 +- 0.034 on 15 Gaussians on a Swiss roll): a reduced copy of that setup
(100 instead of 10,000 samples per distribution, same means) scores within
two reported deviations of those values or above.  That pin is about
rankings only: a wrong recurrence sign or an unhalved b_0 keeps the ranking
(checked by planting them) and is caught by the heat-application pins instead;
a misplaced pair fails the single-pair check.
"""
import numpy as np

import synth
from oracle import graph, pairwise, sinkhorn, spectrum


def test_matrix_places_single_pair_values():
    X = np.random.default_rng(0).standard_normal((30, 3))
    A, info = graph.knn_graph(X, 5)
    L = graph.laplacian(A)
    lam = 1.01 * spectrum.lambda_max(L)
    rng = np.random.default_rng(1)
    H = rng.uniform(0, 1, (30, 4)) * (rng.uniform(0, 1, (30, 4)) < 0.5)
    H /= H.sum(axis=0)
    D = pairwise.distance_matrix(L, lam, 1.0, 20, H, 50)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)
    for i, j in [(0, 1), (1, 3), (2, 3)]:
        ref = sinkhorn.sinkhorn(L, lam, 1.0, 20, H[:, [i]], H[:, [j]], 50, marginals=False)["D"][0]
        assert abs(D[i, j] - ref) <= 1e-12 * max(1.0, abs(ref))
    Dd = pairwise.distance_matrix(L, lam, 1.0, 20, H, 50, diagonal=True)
    ref = sinkhorn.sinkhorn(L, lam, 1.0, 20, H[:, [2]], H[:, [2]], 50, marginals=False)["D"][0]
    assert abs(Dd[2, 2] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_scores_hand_example():
    truth = np.array([[0, 1, 2, 3], [1, 0, 1, 2], [2, 1, 0, 1], [3, 2, 1, 0]], dtype=float)
    s = pairwise.nn_scores(truth, truth, k=1)
    assert s["spearman"] == 1.0 and abs(s["pearson"] - 1.0) < 1e-15 and s["p_at_1"] == 1.0
    rev = 4.0 - truth
    np.fill_diagonal(rev, 0)
    s = pairwise.nn_scores(rev, truth, k=1)
    assert s["spearman"] < 0 and s["pearson"] < 0
    # row 0: nearest under rev is 3, under truth 1; row 1: 3 vs 0 (tie 0/2 -> 0); row 2: 0 vs 1; row 3: 0 vs 2
    assert s["p_at_1"] == 0.0


def test_reduced_swiss_roll_experiment_scores_like_the_paper():
    per = 100
    X, lab, means = synth.gaussians_on_swiss_roll(15, per)
    A, info = graph.knn_graph(X, 10)
    assert info["n_components"] == 1
    L = graph.laplacian(A)
    lam = 1.01 * spectrum.lambda_max(L)
    H = np.zeros((X.shape[0], 15))
    for i in range(15):
        H[lab == i, i] = 1.0 / per
    D = pairwise.distance_matrix(L, lam, 2.0, 30, H, 100)
    truth = np.linalg.norm(means[:, None] - means[None], axis=2)
    s = pairwise.nn_scores(D, truth)
    assert s["spearman"] >= 0.847 - 2 * 0.023, s
    assert s["p_at_5"] >= 0.833 - 2 * 0.034, s


def test_pairs_beyond_K_hops_reduce_to_the_floor_closed_form():
    """Supports more than K hops apart: p_K(L) has exact zeros between them, so
    after the first w-update every denominator on a support floors at phi and
    D = 4t (sum mu ln(mu/phi) + sum nu ln(nu/phi)); floors: |supp nu| in the
    first iteration, |supp mu| + |supp nu| in each later one."""
    n, K, t, J, phi = 400, 20, 1.5, 6, 1e-30
    rp, col, w = synth.cycle_graph(n)
    A = graph.csr_from_arrays(n, rp, col, w)
    L = graph.laplacian(A)
    rng = np.random.default_rng(4)
    mu = np.zeros((n, 2))
    nu = np.zeros((n, 2))
    mu[[0, 1, 2, 3], 0] = rng.dirichlet(np.ones(4))
    nu[[150, 151, 153], 0] = rng.dirichlet(np.ones(3))
    mu[[300, 302], 1] = rng.dirichlet(np.ones(2))
    nu[[100, 101, 102, 103, 104], 1] = rng.dirichlet(np.ones(5))
    out = sinkhorn.sinkhorn(L, 4.0, t, K, mu, nu, J, phi=phi, marginals=False)
    xlx = lambda h: np.sum(np.where(h > 0, h * np.log(np.where(h > 0, h, 1.0) / phi), 0.0), axis=0)
    np.testing.assert_allclose(out["D"], 4 * t * (xlx(mu) + xlx(nu)), rtol=1e-13)
    smu, snu = (mu > 0).sum(), (nu > 0).sum()
    assert out["n_floored"] == snu + (J - 1) * (smu + snu)


def test_total_gradient_matches_finite_differences_of_the_total():
    """G[r, c] against central differences of the total (relative step 1e-4 on H[r, c]),
    with and without the diagonal pairs: a dropped target-side term or a
    diagonal pair counted once fails it."""
    X = np.random.default_rng(2).standard_normal((30, 3))
    A, info = graph.knn_graph(X, 5)
    L = graph.laplacian(A)
    lam = 1.01 * spectrum.lambda_max(L)
    rng = np.random.default_rng(3)
    H = rng.uniform(0.2, 1, (30, 4)) * (rng.uniform(0, 1, (30, 4)) < 0.6)
    H /= H.sum(axis=0)
    t, K, J = 1.0, 20, 30
    coords = [(r, c) for c in range(4) for r in np.flatnonzero(H[:, c] > 0)[:2]]
    for diagonal in (False, True):
        total, G = pairwise.total_gradient(L, lam, t, K, H, J, diagonal=diagonal)
        D = pairwise.distance_matrix(L, lam, t, K, H, J, diagonal=diagonal)
        assert abs(total - np.sum(np.triu(D))) <= 1e-12 * abs(total)
        assert np.all(G[H == 0] == 0)
        for r, c in coords:
            h = 1e-4 * H[r, c]
            Hp, Hm = H.copy(), H.copy()
            Hp[r, c] += h
            Hm[r, c] -= h
            tp = pairwise.total_gradient(L, lam, t, K, Hp, J, diagonal=diagonal)[0]
            tm = pairwise.total_gradient(L, lam, t, K, Hm, J, diagonal=diagonal)[0]
            fd = (tp - tm) / (2 * h)
            assert abs(G[r, c] - fd) <= 1e-6 * max(abs(fd), 1.0), (diagonal, r, c, G[r, c], fd)

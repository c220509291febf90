"""GPU parity of the barycentric distance and the Expected Barycenter Effect.

Parity: gamma within the distance tolerance, both barycenters within 1e-6 L1,
the effect within 1e-5 of the oracle's, on a cluster graph and on the 1-D
graph of the barycenter-effect experiment where one treatment member sits on
a component of its own (floors active on whole components).  Behaviour: on
the synthetic setup of that experiment (control family: 10 x N(0, 1);
treatment: 9 x N(5, 1) plus one shifted member at -60, -30, 0 or 5; 500
samples each, 1-D features, common kNN graph with k = 10), the effect stays
near the true shift 5, nearer to it than the plain difference of sample means
whenever the shifted member is an outlier.  In 1-D a kNN graph with k = 10
splits at any gap wider than the span of ten neighbours; the seed is one whose
graphs split only at the outliers (oracle effect 4.995 at -60 and -30, naive
-1.48 and 1.52; 4.993 at 0, naive 4.518; 5.000 without an outlier).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import families as ofam
from oracle.sinkhorn import barycenter as obary
from gpu_common import lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


def test_barycentric_distance_and_effect_match_oracle(gs):
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    n, K, t, Jb, Js = X.shape[0], 30, 2.0, 40, 60
    rng = np.random.default_rng(31)
    fT, _ = synth.loguniform_support_histograms(n, 4, 30, 800, 1.0, rng)
    fC, _ = synth.loguniform_support_histograms(n, 3, 30, 800, 1.0, rng)
    aT, aC = np.full(4, 0.25), np.array([0.2, 0.3, 0.5])
    lam = lam_hat_of(L)
    gref, pTr, pCr = ofam.barycentric_distance(L, lam, t, K, fT.astype(np.float64), aT, fC.astype(np.float64), aC,
                                               Jb, Js)
    Y = X[:, :3].astype(np.float32)
    tau_ref = ofam.expected_barycenter_effect(pTr, pCr, Y.astype(np.float64))
    g = gs.gs_graph_from_csr(n, *arrs)
    gam, pT, pC = gs.barycentric_distance(g, lam, t, K, to_dev(fT), aT, to_dev(fC), aC, Jb, Js)
    assert abs(gam - gref) <= 1e-5 * max(abs(gref), 4 * t), (gam, gref)
    assert np.abs(to_host(pT) - pTr).sum() <= 1e-6
    assert np.abs(to_host(pC) - pCr).sum() <= 1e-6
    tau = gs.expected_barycenter_effect(pT, pC, to_dev(Y))
    np.testing.assert_allclose(tau, tau_ref, atol=1e-5)


def _effect_setup(shift, seed):
    rng = np.random.default_rng(seed)
    control = [rng.normal(0.0, 1.0, 500) for _ in range(10)]
    treat = [rng.normal(5.0, 1.0, 500) for _ in range(9)] + [rng.normal(shift, 1.0, 500)]
    pts = np.concatenate(control + treat).astype(np.float32)[:, None]
    n = pts.shape[0]
    def indicator(i):
        h = np.zeros(n, dtype=np.float32)
        h[i * 500:(i + 1) * 500] = 1.0 / 500
        return h
    fC = np.stack([indicator(i) for i in range(10)], axis=1)
    fT = np.stack([indicator(10 + i) for i in range(10)], axis=1)
    naive = np.mean(np.concatenate(treat)) - np.mean(np.concatenate(control))
    return pts, fT, fC, naive


def test_barycenters_with_a_disconnected_member_match_oracle(gs):
    pts, fT, fC, naive = _effect_setup(-30.0, seed=12)
    arrs, L, info, A = oracle_csr(pts, 10)
    assert info["n_components"] == 2
    n, K, t, J = pts.shape[0], 30, 2.0, 100
    lam = lam_hat_of(L)
    alpha = np.full(10, 0.1)
    g = gs.gs_graph_from_csr(n, *arrs)
    for fam in (fT, fC):
        ref = obary(L, lam, t, K, fam.astype(np.float64), alpha, J)["p"]
        p = to_host(gs.family_barycenter(g, lam, t, K, to_dev(fam), alpha, J))
        assert np.abs(p - ref).sum() <= 1e-6, np.abs(p - ref).sum()


@pytest.mark.parametrize("shift,n_comp", [(-60.0, 2), (-30.0, 2), (0.0, 1), (5.0, 1)])
def test_expected_barycenter_effect_recovers_the_shift(gs, shift, n_comp):
    pts, fT, fC, naive = _effect_setup(shift, seed=12)
    g = gs.gs_graph_from_points(pts, 10)
    assert g.n_components == n_comp
    lam = gs.gs_lambda_max(g, iters=60, seed=3, safety=1.01)
    K, t = 30, 2.0
    alpha = np.full(10, 0.1)
    pT = gs.family_barycenter(g, lam, t, K, to_dev(fT), alpha, 100)
    pC = gs.family_barycenter(g, lam, t, K, to_dev(fC), alpha, 100)
    tau = float(gs.expected_barycenter_effect(pT, pC, to_dev(pts))[0])
    assert abs(tau - 5.0) < 0.05, tau
    if shift != 5.0:
        assert abs(tau - 5.0) < abs(naive - 5.0), (tau, naive)


@pytest.mark.parametrize("n,d", [(1, 1), (999, 3), (100003, 257), (5000, 4096)])
def test_expectation_matches_float64(gs, n, d):
    """gs_expectation over one or many column tiles (d up to 4096 features),
    ragged n, a single node: float64 products and fixed-order sums, so within
    1e-12 of the float64 weighted mean of the same float32 inputs; a signal of
    zero mass is refused with GS_ERR_NONFINITE."""
    rng = np.random.default_rng(n + d)
    p = (rng.uniform(0.0, 1.0, n) * (rng.uniform(size=n) < 0.5)).astype(np.float32)
    p[0] = 0.75
    Y = rng.standard_normal((n, d)).astype(np.float32)
    got = gs.gs_expectation(to_dev(p), to_dev(Y))
    p64, Y64 = p.astype(np.float64), Y.astype(np.float64)
    ref = (p64 @ Y64) / p64.sum()
    scale = (p64 @ np.abs(Y64)) / p64.sum()
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300), np.abs(got - ref).max()
    with pytest.raises(gs.GeoSinkError) as e:
        gs.gs_expectation(torch.zeros(n, device="cuda"), to_dev(Y))
    assert e.value.status == -6

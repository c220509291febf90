"""The graph-level calls (gs_graph_heat_apply, gs_graph_sinkhorn,
gs_graph_sinkhorn_backward, gs_graph_barycenter): the same computation as
the plan-bound calls they wrap, bit for bit against a plan created with the
same (graph, K, B) and default flags, which is what the graph keeps when no
plan is given; the heat application also against the float64 oracle; a
caller's plan for another K or B is refused; the kept plans go with the
graph.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import heat
from gpu_common import heat_tol, lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def curve():
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    return X.shape[0], labels, arrs, L


def bits(t):
    return t.detach().contiguous().view(torch.int32).cpu()


def pairs(labels, seed, B):
    rng = np.random.default_rng(seed)
    ps = [synth.cluster_block_pair(labels, s, 2, 1.0, rng) for s in range(0, 2 * B, 2)]
    return (np.stack([p[0] for p in ps], axis=1).astype(np.float32),
            np.stack([p[1] for p in ps], axis=1).astype(np.float32))


def test_heat_apply_graph_level(gs, curve):
    n, labels, arrs, L = curve
    g = gs.gs_graph_from_csr(n, *arrs)
    lam, t, K, B = lam_hat_of(L), 1.5, 20, 8
    x = synth.random_dense_like(n, B, np.random.default_rng(3))
    Y0, Y1, D0, D1 = (torch.empty(n * B, device="cuda") for _ in range(4))
    plan = gs.Plan(g, K, B)
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y0, D0)
    gs.gs_graph_heat_apply(g, lam, t, K, to_dev(x), Y1, D1)
    assert torch.equal(bits(Y0), bits(Y1)) and torch.equal(bits(D0), bits(D1))
    ref = heat.heat_apply(L, lam, t, K, x.astype(np.float64))
    assert np.abs(to_host(Y1).reshape(n, B) - ref).max() <= heat_tol(K, np.abs(x).max())
    Y2 = torch.empty(n * B, device="cuda")
    gs.gs_graph_heat_apply(g, lam, t, K, to_dev(x), Y2, plan=plan)   # the caller's plan
    assert torch.equal(bits(Y0), bits(Y2))


@pytest.mark.parametrize("ce", [4, -1])
def test_sinkhorn_and_reverse_sweep_graph_level(gs, curve, ce):
    n, labels, arrs, L = curve
    g = gs.gs_graph_from_csr(n, *arrs)
    lam, t, K, J, B = lam_hat_of(L), 2.0, 12, 10, 4
    mu, nu = pairs(labels, 5, B)
    mud, nud = to_dev(mu), to_dev(nu)
    a = to_dev(np.random.default_rng(6).uniform(0.5, 1.5, n))
    ce = gs.GS_RECORD_ALL if ce < 0 else ce
    plan = gs.Plan(g, K, B)
    res = []
    for graph_level in (False, True):
        v, w = torch.empty(n * B, device="cuda"), torch.empty(n * B, device="cuda")
        ck = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
        gm, gn = torch.empty(n * B, device="cuda"), torch.empty(n * B, device="cuda")
        if graph_level:
            out = gs.gs_graph_sinkhorn(g, lam, t, K, mud, nud, J, a=a, ckpt_every=ce, ckpt=ck, v=v, w=w,
                                       want_marg=True, want_floors=True)
            gt = gs.gs_graph_sinkhorn_backward(g, lam, t, K, mud, nud, J, ce, ck, np.ones(B), a=a, grad_mu=gm,
                                               grad_nu=gn)
        else:
            out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, a=a, ckpt_every=ce, ckpt=ck, v=v, w=w, want_marg=True,
                                 want_floors=True)
            gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ck, np.ones(B), a=a, grad_mu=gm, grad_nu=gn)
        res.append((out, v, w, gm, gn, gt))
    (o0, *t0, gt0), (o1, *t1, gt1) = res
    assert np.array_equal(o0["dist"], o1["dist"]) and np.array_equal(o0["marg_err"], o1["marg_err"])
    assert o0["n_floored"] == o1["n_floored"]
    for x0, x1 in zip(t0, t1):
        assert torch.equal(bits(x0), bits(x1))
    assert np.array_equal(gt0, gt1)


def test_barycenter_graph_level(gs, curve):
    n, labels, arrs, L = curve
    g = gs.gs_graph_from_csr(n, *arrs)
    lam, t, K, J, m = lam_hat_of(L), 2.0, 15, 25, 6
    H, _ = synth.loguniform_support_histograms(n, m, 30, 1500, 0.5, np.random.default_rng(3))
    alpha = np.full(m, 1.0 / m)
    plan = gs.Plan(g, K, m)
    b0, b1 = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    o0 = gs.gs_barycenter(plan, lam, t, to_dev(H), alpha, J, b0, want_marg=True)
    o1 = gs.gs_graph_barycenter(g, lam, t, K, to_dev(H), alpha, J, b1, want_marg=True)
    assert torch.equal(bits(b0), bits(b1)) and np.array_equal(o0["marg_err"], o1["marg_err"])


def test_foreign_plans_are_refused_and_kept_plans_go_with_the_graph(gs, curve):
    n, labels, arrs, L = curve
    g = gs.gs_graph_from_csr(n, *arrs)
    other = gs.gs_graph_from_csr(n, *arrs)
    lam, t = lam_hat_of(L), 1.0
    x = to_dev(synth.random_dense_like(n, 4, np.random.default_rng(1)))
    Y = torch.empty(n * 4, device="cuda")
    for plan in (gs.Plan(g, 9, 4), gs.Plan(g, 10, 8), gs.Plan(other, 10, 4)):
        with pytest.raises(gs.GeoSinkError, match="plan was created for another graph, K or B"):
            gs.gs_graph_heat_apply(g, lam, t, 10, x, Y, plan=plan)
    for K in (5, 10, 5):   # two kept plans, the first reused
        gs.gs_graph_heat_apply(g, lam, t, K, x, Y)
    torch.cuda.synchronize()
    g.destroy()   # frees the kept plans
    other.destroy()
    torch.cuda.synchronize()

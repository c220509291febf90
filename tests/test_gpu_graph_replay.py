"""Captured hipGraphs against direct launches, over repeated calls.

Every driver captures its iterations in hipGraphs on first use and replays
them on later calls (one graph per chunk of recorded iterations, per
checkpoint segment, per reverse iteration).  Each call below runs three times
per plan, with unrelated eager work and a synchronisation between the calls,
once with graphs and once with GS_PLAN_NO_GRAPH (the same kernels launched
directly): every output of every call is bitwise equal to the first direct
call's.  Sizes: a 2000-node local graph with hub rows (long-row blocks in
every launch), J = 7 (checkpoint segments of 3, 3, 1), B = 1 and B = 6 (a
padded row of 8 floats).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def graph(gs):
    n = 2000
    arrs = synth.random_local_graph(n, 6, 200, np.random.default_rng(31), hubs=2, hub_degree=900)
    return gs.gs_graph_from_csr(n, *arrs), n


def _eager_noise():
    a = torch.randn(1 << 20, device="cuda")
    (a * 2.0 + 1.0).sum().item()
    torch.cuda.synchronize()


def _sinkhorn_outputs(gs, plan, n, B, lam, t, J, ce, mu, nu):
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    v = torch.empty(n * B, device="cuda")
    w = torch.empty(n * B, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mu, nu, J, ckpt_every=ce, ckpt=ckpt, v=v, w=w, want_marg=True,
                         want_floors=True)
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, ce, ckpt, np.linspace(1.0, 2.0, B), grad_mu=gmu,
                                 grad_nu=gnu)
    torch.cuda.synchronize()
    return [out["dist"], out["marg_err"], np.array([out["n_floored"]]), v.cpu().numpy(), w.cpu().numpy(),
            gmu.cpu().numpy(), gnu.cpu().numpy(), gt]


@pytest.mark.parametrize("B", [1, 6])
@pytest.mark.parametrize("ce", [-1, 3])
def test_sinkhorn_and_reverse_sweep_replays(gs, graph, B, ce):
    g, n = graph
    K, t, J = 20, 1.5, 7
    lam = g.edge_bound
    rng = np.random.default_rng(B * 10 + ce)
    mu = to_dev(synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.3))
    nu = to_dev(synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.3))
    runs = []
    for flags in (gs.GS_PLAN_NO_GRAPH, 0):
        plan = gs.Plan(g, K, B, flags=flags)
        for _ in range(3):
            runs.append(_sinkhorn_outputs(gs, plan, n, B, lam, t, J, ce, mu, nu))
            _eager_noise()
    ref = runs[0]
    assert all(np.all(np.isfinite(x)) for x in ref)
    for r in runs[1:]:
        for a, b in zip(ref, r):
            assert np.array_equal(a, b)


def test_barycenter_replays(gs, graph):
    g, n = graph
    K, t, J, m = 20, 1.5, 6, 5
    lam = g.edge_bound
    rng = np.random.default_rng(41)
    mus = to_dev(synth.random_dense_like(n, m, rng, positive=True) * (rng.uniform(size=(n, m)) < 0.4))
    alpha = rng.dirichlet(np.ones(m))
    runs = []
    for flags in (gs.GS_PLAN_NO_GRAPH, 0):
        plan = gs.Plan(g, K, m, flags=flags)
        for _ in range(3):
            p = torch.empty(n, device="cuda")
            out = gs.gs_barycenter(plan, lam, t, mus, alpha, J, p, want_marg=True, want_floors=True)
            torch.cuda.synchronize()
            runs.append([p.cpu().numpy(), out["marg_err"], np.array([out["n_floored"]])])
            _eager_noise()
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)

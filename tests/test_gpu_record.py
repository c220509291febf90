"""Record mode of Algorithm 1's reverse sweep (ckpt_every = GS_RECORD_ALL).

The forward keeps every iteration's floored denominators, so the reverse
sweep recomputes nothing.  Against the checkpointed sweep (which the oracle
tests check): distances, v, w and floor counts are bitwise equal, the
gradients in mu and nu bitwise equal, the gradient in t equal up to the
rounding of the first reduction of each checkpoint segment (the
checkpointed sweep reads the stored w there, the record sweep nu / e), for
ragged and full widths, with and without vertex weights, with J not a
multiple of the graph chunk or the checkpoint interval, and again on a
second record buffer (captured graphs hold the buffer's address).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def swiss():
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    arrs, L, info, A = oracle_csr(X, 10)
    return arrs, L


def _run(gs, plan, lam, t, mu, nu, J, ce, a):
    n, B = mu.shape
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    v = torch.empty(n * B, device="cuda")
    w = torch.empty(n * B, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mu, nu, J, a=a, ckpt_every=ce, ckpt=ckpt, v=v, w=w, want_floors=True)
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gd = np.linspace(0.5, 1.5, B)
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, ce, ckpt, gd, a=a, grad_mu=gmu, grad_nu=gnu)
    return out, v, w, gmu, gnu, gt


@pytest.mark.parametrize("B", [3, 32])
@pytest.mark.parametrize("weighted", [False, True])
def test_record_mode_equals_checkpointed_sweep(gs, swiss, B, weighted):
    arrs, L = swiss
    n, K, t, J = 2000, 20, 1.0, 21
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    rng = np.random.default_rng(B + 7 * weighted)
    mu = np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1)
    nu = np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1)
    a = to_dev(rng.uniform(0.5, 1.5, n).astype(np.float32)) if weighted else None
    mud, nud = to_dev(mu), to_dev(nu)
    plan = gs.Plan(g, K, B)
    ref = _run(gs, plan, lam, t, mud, nud, J, 5, a)
    for again in range(2):          # second pass: a new record buffer
        rec = _run(gs, plan, lam, t, mud, nud, J, gs.GS_RECORD_ALL, a)
        assert np.array_equal(rec[0]["dist"], ref[0]["dist"])
        assert rec[0]["n_floored"] == ref[0]["n_floored"]
        for i in (1, 2, 3, 4):
            assert torch.equal(rec[i], ref[i]), (again, i)
        np.testing.assert_allclose(rec[5], ref[5], rtol=1e-6, atol=1e-6 * np.abs(ref[5]).max())


def test_record_mode_single_iteration(gs, swiss):
    """J = 1: one record chunk of one iteration; the sweep's only reduction uses w^0 = 1."""
    arrs, L = swiss
    n, K, t, J, B = 2000, 20, 1.0, 1, 3
    g = gs.gs_graph_from_csr(n, *arrs)
    rng = np.random.default_rng(77)
    mu = np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1)
    nu = np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1)
    plan = gs.Plan(g, K, B)
    ref = _run(gs, plan, lam_hat_of(L), t, to_dev(mu), to_dev(nu), J, 1, None)
    rec = _run(gs, plan, lam_hat_of(L), t, to_dev(mu), to_dev(nu), J, gs.GS_RECORD_ALL, None)
    assert np.array_equal(rec[0]["dist"], ref[0]["dist"])
    for i in (1, 2, 3, 4):
        assert torch.equal(rec[i], ref[i]), i
    np.testing.assert_allclose(rec[5], ref[5], rtol=1e-6, atol=1e-6 * np.abs(ref[5]).max())


@pytest.mark.parametrize("ce", [-1, 5])
def test_histogram_gradients_without_grad_t_are_bitwise_equal(gs, swiss, ce):
    """grad_t = NULL runs plain adjoint applications instead of the dual form
    and skips the t reductions; grad_mu and grad_nu are bitwise those of the
    sweep that also forms grad_t (records and checkpoint segments), also
    when the two kinds of call alternate on one plan (separate captured graphs)."""
    arrs, L = swiss
    n, K, t, J, B = 2000, 20, 1.0, 13, 6
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    rng = np.random.default_rng(91)
    mu = to_dev(np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1))
    nu = to_dev(np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1))
    a = to_dev(rng.uniform(0.5, 1.5, n).astype(np.float32))
    plan = gs.Plan(g, K, B)
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    gs.gs_sinkhorn(plan, lam, t, mu, nu, J, a=a, ckpt_every=ce, ckpt=ckpt)
    gd = np.linspace(0.5, 1.5, B)
    outs = []
    for want_t in (True, False, True, False):
        gmu = torch.empty(n * B, device="cuda")
        gnu = torch.empty(n * B, device="cuda")
        gt = gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, ce, ckpt, gd, a=a, grad_mu=gmu, grad_nu=gnu,
                                     want_grad_t=want_t)
        assert (gt is not None) == want_t
        outs.append((gmu, gnu, gt))
    for gmu, gnu, _ in outs[1:]:
        assert torch.equal(gmu, outs[0][0]) and torch.equal(gnu, outs[0][1])
    assert np.array_equal(outs[0][2], outs[2][2])


def test_growing_checkpoint_interval_on_one_plan(gs, swiss):
    """A plan first used with checkpoints every 5 iterations (J = 5: one
    captured segment of length 5), then every 10 with J = 15 (segments of 10
    and 5): the segment buffers grow, and the second sweep must not replay
    graphs captured over the old buffers.  Its results are bitwise those of a
    fresh plan running only the second configuration."""
    arrs, L = swiss
    n, K, t, B = 2000, 20, 1.0, 4
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = lam_hat_of(L)
    rng = np.random.default_rng(123)
    mu = to_dev(np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1))
    nu = to_dev(np.stack([synth.uniform_on_random_nodes(n, 400, rng) for _ in range(B)], axis=1))
    reused = gs.Plan(g, K, B)
    _run(gs, reused, lam, t, mu, nu, 5, 5, None)
    got = _run(gs, reused, lam, t, mu, nu, 15, 10, None)
    ref = _run(gs, gs.Plan(g, K, B), lam, t, mu, nu, 15, 10, None)
    assert np.array_equal(got[0]["dist"], ref[0]["dist"])
    for i in (1, 2, 3, 4):
        assert torch.equal(got[i], ref[i]), i
    assert np.array_equal(got[5], ref[5])

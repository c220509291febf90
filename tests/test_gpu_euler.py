"""GPU parity of the backward-Euler heat kernel (I + (t/N) L_op)^{-N} by CG.

Against the oracle's exact sparse solves: heat applications over several
widths (ragged included), step counts and times; Algorithm 1 and the
barycenter with this kernel; the 1M-node cycle against its Fourier closed
form.  Tolerance of an application, per column in the 2-norm: each solve
stops at the CG bound 2^-52 ||b|| plus float32 rounding of order m kappa u ||b||
(m iterations, kappa <= 1 + 2t/N, u = 2^-24), and later solves do not amplify
earlier errors (||(I + cL)^{-1}|| <= 1), so N solves stay within
N (2^-52 + 4 m kappa u) ||x||.  Algorithm 1 with this kernel matches the
oracle's exact solves only because the automatic count drives the CG bound far
below float32 resolution (with the bound at 1e-7, 8 instead of 17 iterations
at kappa = 1.5, distances differ by 7e-3, the same in a float64 emulation).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms, heat, sinkhorn
from gpu_common import lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


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


def cg_count(t, N):
    sk = math.sqrt(1 + 2 * t / N)
    rho = (sk - 1) / (sk + 1)
    return max(1, math.ceil(math.log(2 * sk / 2.0 ** -52) / math.log(1 / rho)))


def euler_tol(t, N, x):
    kappa = 1 + 2 * t / N
    return N * (2.0 ** -52 + 4 * cg_count(t, N) * kappa * U) * np.linalg.norm(x, axis=0)


@pytest.mark.parametrize("B", [1, 3, 32])
@pytest.mark.parametrize("N,t", [(1, 0.5), (1, 2.0), (4, 2.0), (10, 2.0), (10, 8.0)])
def test_euler_apply_matches_oracle(gs, swiss, B, N, t):
    arrs, L = swiss
    n = 2000
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    x = synth.random_dense_like(n, B, np.random.default_rng(10 * B + N))
    plan = gs.Plan(g, 4, B)
    plan.set_kernel(gs.GS_KERNEL_EULER, N)
    assert "kernel=euler" in plan.describe()
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = heat.euler_apply(L, lam, t, N, x.astype(np.float64))
    err = np.linalg.norm(to_host(Y).reshape(n, B) - ref, axis=0)
    tol = euler_tol(t, N, x.astype(np.float64))
    print("euler", B, N, t, (err / np.linalg.norm(x, axis=0)).max())
    assert np.all(err <= tol), (err, tol)


def test_euler_sinkhorn_and_barycenter_match_oracle(gs, swiss):
    arrs, L = swiss
    n, N, t, J, B = 2000, 4, 1.0, 60, 4
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    rng = np.random.default_rng(3)
    mu = np.stack([synth.uniform_on_random_nodes(n, 300, rng) for _ in range(B)], axis=1)
    nu = np.stack([synth.uniform_on_random_nodes(n, 300, rng) for _ in range(B)], axis=1)
    E = lambda v: heat.euler_apply(L, lam, t, N, v)
    ref = sinkhorn.sinkhorn(L, lam, t, 0, mu.astype(np.float64), nu.astype(np.float64), J, apply=E,
                            marginals=False)
    plan = gs.Plan(g, 4, B)
    plan.set_kernel(gs.GS_KERNEL_EULER, N)
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, want_floors=True)
    print("euler sinkhorn", np.abs(out["dist"] - ref["D"]).max(), ref["D"])
    assert np.all(np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t))
    assert out["n_floored"] == ref["n_floored"]
    alpha = np.full(B, 1.0 / B)
    pref = sinkhorn.barycenter(L, lam, t, 0, mu.astype(np.float64), alpha, 40, apply=E)["p"]
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, to_dev(mu), alpha, 40, bary)
    print("euler bary", np.abs(to_host(bary) - pref).sum())
    assert np.abs(to_host(bary) - pref).sum() <= 1e-6


def test_euler_sinkhorn_with_vertex_weights(gs, swiss):
    """Vertex weights a go through the scaling epilogue (out_a = a out) of the Euler form."""
    arrs, L = swiss
    n, N, t, J, B = 2000, 3, 0.8, 40, 2
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    rng = np.random.default_rng(17)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    mu = np.stack([synth.uniform_on_random_nodes(n, 250, rng) for _ in range(B)], axis=1)
    nu = np.stack([synth.uniform_on_random_nodes(n, 250, rng) for _ in range(B)], axis=1)
    E = lambda v: heat.euler_apply(L, lam, t, N, v)
    ref = sinkhorn.sinkhorn(L, lam, t, 0, mu.astype(np.float64), nu.astype(np.float64), J,
                            a=a.astype(np.float64), apply=E, marginals=False)
    plan = gs.Plan(g, 4, B)
    plan.set_kernel(gs.GS_KERNEL_EULER, N)
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, a=to_dev(a))
    assert np.all(np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t))


def test_euler_graph_replay_and_switch_back(gs, swiss):
    arrs, L = swiss
    n, B = 2000, 8
    lam = lam_hat_of(L)
    g = gs.gs_graph_from_csr(n, *arrs)
    xd = to_dev(synth.random_dense_like(n, B, np.random.default_rng(1)))
    outs = []
    for flags in (0, gs.GS_PLAN_NO_GRAPH):
        plan = gs.Plan(g, 10, B, flags=flags)
        plan.set_kernel(gs.GS_KERNEL_EULER, 3, 0)
        Y = torch.empty(n * B, device="cuda")
        for _ in range(3):
            gs.gs_heat_apply(plan, lam, 2.0, xd, Y)
            torch.cuda.synchronize()
            outs.append(Y.clone())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    plan = gs.Plan(g, 10, B)
    fresh = gs.Plan(g, 10, B)
    plan.set_kernel(gs.GS_KERNEL_EULER, 3, 5)
    Y = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, 2.0, xd, Y)
    plan.set_kernel(gs.GS_KERNEL_CHEBYSHEV)
    Yc, Yf = torch.empty_like(Y), torch.empty_like(Y)
    gs.gs_heat_apply(plan, lam, 2.0, xd, Yc)
    gs.gs_heat_apply(fresh, lam, 2.0, xd, Yf)
    assert torch.equal(Yc, Yf)


def test_euler_rejects_derivative_and_reverse_sweep(gs, swiss):
    arrs, L = swiss
    n, B = 2000, 2
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, 10, B)
    plan.set_kernel(gs.GS_KERNEL_EULER, 2)
    x = torch.ones(n * B, device="cuda")
    Y, Yd = torch.empty_like(x), torch.empty_like(x)
    with pytest.raises(gs.GeoSinkError):
        gs.gs_heat_apply(plan, 10.0, 1.0, x, Y, Yd)
    ckpt = torch.empty(gs.n_checkpoints(4, 2) * n * B, device="cuda")
    with pytest.raises(gs.GeoSinkError):
        gs.gs_sinkhorn_backward(plan, 10.0, 1.0, x / n, x / n, 4, 2, ckpt, np.ones(B))
    with pytest.raises(gs.GeoSinkError):
        plan.set_kernel(gs.GS_KERNEL_EULER, 0)


@pytest.mark.parametrize("N", [1, 5])
def test_euler_cycle_one_million_nodes_closed_form(gs, N):
    n, t, lam = 1_000_000, 2.0, 4.0
    g = gs.gs_graph_from_csr(n, *synth.cycle_graph(n))
    x = synth.random_dense_like(n, 1, np.random.default_rng(N))
    plan = gs.Plan(g, 4, 1)
    plan.set_kernel(gs.GS_KERNEL_EULER, N)
    Y = torch.empty(n, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Y)
    ref = closed_forms.cycle_euler_apply(n, lam, t, N, x.astype(np.float64))
    err = np.linalg.norm(to_host(Y).reshape(n, 1) - ref, axis=0)
    assert np.all(err <= euler_tol(t, N, x.astype(np.float64))), err

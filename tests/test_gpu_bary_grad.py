"""GPU parity of the barycenter iteration and of the hand-written backward.

Barycenter: ||p_gpu - p_ref||_1 <= 1e-6.  Gradients: ||g - g_ref||_2 /
||g_ref||_2 <= 1e-4 on the supports, and sampled coordinates within 1e-4 of
max(|g_ref_i|, 1e-3 ||g_ref||_inf); the t-gradient within 1e-4 relative.
The per-coordinate floor: float32 gradient entries carry an absolute error
of a few u * ||g||_inf (u = 2^-24, entries are sums of 4t ln v terms of size
up to ||g||_inf), so a coordinate that cancels to near zero cannot be
accurate to 1e-4 of itself; 1e-4 * 1e-3 ||g||_inf = 1e-7 ||g||_inf is ~1.7 u.
The tests print the worst ratio with both the 1e-3 floor and a 1e-2 floor.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import heat
from oracle import sinkhorn as osk
from gpu_common import csr_laplacian, lam_hat_of, need_gpu, oracle_csr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


@pytest.fixture(scope="module")
def clusters():
    X, labels = synth.clusters_on_curve(10, 300, dim=50, sigma=0.1, workload=3)
    arrs, L, info, A = oracle_csr(X, 15)
    assert info["n_components"] == 1
    return X.shape[0], labels, arrs, L


def test_barycenter_matches_oracle(gs, clusters):
    """Reduced twin of the batched barycenter workload: m = 8 inputs, Dirichlet(0.5), K = 40, t = 2."""
    n, labels, arrs, L = clusters
    m, K, t, J = 8, 40, 2.0, 40
    rng = np.random.default_rng(synth.seed_for(3, 2))
    H, _ = synth.loguniform_support_histograms(n, m, 30, 1500, 0.5, rng)
    alpha = np.full(m, 1.0 / m)
    lam = lam_hat_of(L)
    ref = osk.barycenter(L, lam, t, K, H.astype(np.float64), alpha, J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, m)
    bary = torch.empty(n, device="cuda")
    out = gs.gs_barycenter(plan, lam, t, to_dev(H), alpha, J, bary, want_marg=True, want_floors=True)
    p = to_host(bary)
    assert np.abs(p - ref["p"]).sum() <= 1e-6, np.abs(p - ref["p"]).sum()
    assert out["n_floored"] == ref["n_floored"]
    np.testing.assert_allclose(out["marg_err"], ref["marg_row"], rtol=0.05, atol=2e-7)


def test_barycenter_with_vertex_weights_matches_oracle(gs, clusters):
    """Vertex weights a (R7) in the barycenter iteration: m = 5 inputs, K = 30, t = 1."""
    n, labels, arrs, L = clusters
    m, K, t, J = 5, 30, 1.0, 30
    rng = np.random.default_rng(71)
    H, _ = synth.loguniform_support_histograms(n, m, 30, 1500, 0.5, rng)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    alpha = np.array([0.1, 0.2, 0.3, 0.25, 0.15])
    lam = lam_hat_of(L)
    ref = osk.barycenter(L, lam, t, K, H.astype(np.float64), alpha, J, a=a.astype(np.float64))
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, m)
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, to_dev(H), alpha, J, bary, a=to_dev(a))
    assert np.abs(to_host(bary) - ref["p"]).sum() <= 1e-6, np.abs(to_host(bary) - ref["p"]).sum()


def test_barycenter_single_input_is_smoothed_input(gs, clusters):
    n, labels, arrs, L = clusters
    K, t = 30, 1.0
    rng = np.random.default_rng(8)
    H, _ = synth.loguniform_support_histograms(n, 1, 100, 400, 1.0, rng)
    lam = lam_hat_of(L)
    ref = osk.barycenter(L, lam, t, K, H.astype(np.float64), np.array([1.0]), 3)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, to_dev(H), [1.0], 3, bary)
    assert np.abs(to_host(bary) - ref["p"]).sum() <= 1e-6


def test_barycenter_one_hot_weights_ignore_the_other_inputs(gs, clusters):
    """alpha = e_2 among m = 5 inputs: p = q_2 after one iteration, w_2 = 1,
    so p stays p_K mu_2 / p_K(0) (the single-input closed form) whatever the
    other inputs are; also against the oracle's iteration."""
    n, labels, arrs, L = clusters
    m, K, t, J = 5, 30, 1.0, 4
    rng = np.random.default_rng(18)
    H, _ = synth.loguniform_support_histograms(n, m, 100, 400, 1.0, rng)
    alpha = np.zeros(m)
    alpha[2] = 1.0
    lam = lam_hat_of(L)
    ref = osk.barycenter(L, lam, t, K, H.astype(np.float64), alpha, J)
    b = heat.cheb_coeffs(t, K)
    p0 = b[0] / 2 + sum((-1) ** k * b[k] for k in range(1, K + 1))
    closed = heat.heat_apply(L, lam, t, K, H[:, 2].astype(np.float64)) / p0
    assert np.abs(ref["p"] - closed).sum() <= 1e-12
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, m)
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, to_dev(H), alpha, J, bary)
    assert np.abs(to_host(bary) - closed).sum() <= 1e-6


@pytest.mark.parametrize("B", [1, 6])
def test_hub_rows_forward_and_backward(gs, B):
    """Rows with 1500-2900 nonzeros run in the long-row blocks: Algorithm 1's
    scaling epilogue (the floor counter runs over a partial wave; supports on
    a third of the nodes leave nothing to floor, as in the oracle) and the
    dual adjoint step there, against the oracle."""
    n, K, t, J = 6000, 12, 1.0, 4
    arrs = synth.random_local_graph(n, 6, 300, np.random.default_rng(21), hubs=4, hub_degree=2900)
    assert np.diff(arrs[0]).max() > 1500
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    rng = np.random.default_rng(30 + B)
    mu = synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.33)
    nu = synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.33)
    mu /= mu.sum(axis=0)
    nu /= nu.sum(axis=0)
    gd = np.linspace(1.0, 2.0, B)
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, g=gd)
    fl = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, marginals=False)["n_floored"]
    plan = gs.Plan(g, K, B)
    mud, nud = to_dev(mu), to_dev(nu)
    ckpt = torch.empty(gs.ckpt_floats(plan, J, gs.GS_RECORD_ALL), device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=gs.GS_RECORD_ALL, ckpt=ckpt, want_floors=True)
    assert out["n_floored"] == fl
    assert (np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)).all(), (out["dist"], ref["D"])
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, gs.GS_RECORD_ALL, ckpt, gd, grad_mu=gmu, grad_nu=gnu)
    for got, want, h in ((to_host(gmu).reshape(n, B), ref["dmu"], mu), (to_host(gnu).reshape(n, B), ref["dnu"], nu)):
        for b in range(B):
            s_ = h[:, b] > 0
            rel = np.linalg.norm(got[s_, b] - want[s_, b]) / np.linalg.norm(want[s_, b])
            assert rel <= 1e-4, (b, rel)
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)


def test_hub_row_floors_are_counted(gs):
    """A floored hub row: a local banded graph plus one hub (2005 nonzeros,
    a long-row block) linked to nodes 3000-4999, mu around the hub, nu on
    nodes 0-50, K = 5: every denominator on either support is a structural
    zero after the first v-update, so the counts (long-row and ordinary
    blocks, partial-wave ballots) must equal the oracle's exactly, and D its
    floor value."""
    import scipy.sparse as sp
    n, hub, B, K, t, J = 6000, 5000, 2, 5, 1.0, 3
    rp, col, w = synth.random_local_graph(n, 3, 10, np.random.default_rng(40))
    A = sp.csr_matrix((w.astype(np.float64), col, rp), shape=(n, n))
    nb = np.arange(3000, 5000)
    H = sp.coo_matrix((np.full(len(nb), 0.5), (np.full(len(nb), hub), nb)), shape=(n, n))
    A2 = (A + H + H.T).tocsr()
    A2.sort_indices()
    arrs = (A2.indptr.astype(np.int32), A2.indices.astype(np.int32), A2.data.astype(np.float32))
    assert np.diff(arrs[0])[hub] > 1500
    L = csr_laplacian(n, arrs)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    rng = np.random.default_rng(41)
    mu = np.zeros((n, B), dtype=np.float32)
    nu = np.zeros((n, B), dtype=np.float32)
    mu[4990:5011] = rng.uniform(0.1, 1.0, (21, B))
    nu[0:51] = rng.uniform(0.1, 1.0, (51, B))
    mu /= mu.sum(axis=0)
    nu /= nu.sum(axis=0)
    ref = osk.sinkhorn(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, marginals=False)
    assert ref["n_floored"] == B * ((J - 1) * 21 + J * 51)
    plan = gs.Plan(g, K, B)
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J, want_floors=True)
    assert out["n_floored"] == ref["n_floored"]
    assert (np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)).all(), (out["dist"], ref["D"])


def _grad_case(n, labels, B, rng):
    mus, nus = [], []
    for b in range(B):
        s = int(rng.integers(0, 6))
        mu, nu = synth.cluster_block_pair(labels, s, 2, 1.0, rng)
        mus.append(mu)
        nus.append(nu)
    return np.stack(mus, axis=1), np.stack(nus, axis=1)


@pytest.mark.parametrize("J,ce", [(20, 10), (23, 10), (12, 5)])
def test_backward_matches_oracle_reverse_mode(gs, clusters, J, ce):
    """Batched pairs on adjacent cluster blocks, K = 30, t = 2; segments of ce iterations."""
    n, labels, arrs, L = clusters
    B, K, t = 4, 30, 2.0
    rng = np.random.default_rng(J * 7 + ce)
    mu, nu = _grad_case(n, labels, B, rng)
    gd = np.array([1.0, -0.5, 2.0, 0.25])
    lam = lam_hat_of(L)
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, g=gd)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    ckpt = torch.empty(gs.n_checkpoints(J, ce) * n * B, device="cuda")
    mud, nud = to_dev(mu), to_dev(nu)
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=ce, ckpt=ckpt)
    assert (np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)).all()
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ckpt, gd, grad_mu=gmu, grad_nu=gnu)
    worst = {1e-3: 0.0, 1e-2: 0.0}
    for got, want, h in ((to_host(gmu).reshape(n, B), ref["dmu"], mu), (to_host(gnu).reshape(n, B), ref["dnu"], nu)):
        for b in range(B):
            s = h[:, b] > 0
            assert np.all(got[~s, b] == 0)
            rel = np.linalg.norm(got[s, b] - want[s, b]) / np.linalg.norm(want[s, b])
            assert rel <= 1e-4, (b, rel)
            idx = np.nonzero(s)[0][:: max(1, s.sum() // 16)][:16]
            for fl in worst:
                scale = np.maximum(np.abs(want[idx, b]), fl * np.abs(want[s, b]).max())
                worst[fl] = max(worst[fl], float(np.max(np.abs(got[idx, b] - want[idx, b]) / scale)))
    # sampled coordinates: |g - g_ref| / max(|g_ref,i|, floor ||g_ref||_inf), both floors reported
    print(f"J={J} ce={ce}: worst sampled-coordinate error / max(|g_i|, 1e-3 ||g||_inf) = {worst[1e-3]:.2e}, "
          f"with 1e-2 ||g||_inf = {worst[1e-2]:.2e}")
    assert worst[1e-3] <= 1e-4
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)


@pytest.mark.parametrize("zeros", [False, True])
@pytest.mark.parametrize("ce", [7, -1])
def test_backward_with_vertex_weights_matches_oracle(gs, clusters, ce, zeros):
    """Vertex weights a (R7) through forward and reverse sweep, checkpointed and
    recorded; also with a = 0 on a tenth of the nodes (allowed: a >= 0)."""
    n, labels, arrs, L = clusters
    B, K, t, J = 3, 30, 1.5, 15
    rng = np.random.default_rng(55)
    mu, nu = _grad_case(n, labels, B, rng)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    if zeros:
        a[rng.choice(n, n // 10, replace=False)] = 0.0
    lam = lam_hat_of(L)
    gd = np.array([1.0, -0.7, 0.4])
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J,
                            a=a.astype(np.float64), g=gd)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    mud, nud, ad = to_dev(mu), to_dev(nu), to_dev(a)
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, a=ad, ckpt_every=ce, ckpt=ckpt)
    assert (np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)).all()
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ckpt, gd, a=ad, grad_mu=gmu, grad_nu=gnu)
    for got, want, h in ((to_host(gmu).reshape(n, B), ref["dmu"], mu), (to_host(gnu).reshape(n, B), ref["dnu"], nu)):
        for b in range(B):
            s_ = h[:, b] > 0
            rel = np.linalg.norm(got[s_, b] - want[s_, b]) / np.linalg.norm(want[s_, b])
            assert rel <= 1e-4, (b, rel)
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)


def test_gradient_matches_fp64_finite_differences(gs, clusters):
    """The GPU gradient (record mode) against central differences of the float64
    oracle's forward: 16 random support coordinates of mu with relative step
    1e-4, and t with step 1e-4 (one pair, K = 30, t = 2, J = 20)."""
    n, labels, arrs, L = clusters
    K, t, J = 30, 2.0, 20
    rng = np.random.default_rng(123)
    mu, nu = _grad_case(n, labels, 1, rng)
    lam = lam_hat_of(L)
    m64, n64 = mu[:, 0].astype(np.float64), nu[:, 0].astype(np.float64)
    coords = rng.choice(np.nonzero(m64 > 0)[0], size=16, replace=False)
    fd = osk.finite_diff_mu(L, lam, t, K, m64, n64, J, coords)
    fdt = osk.finite_diff_t(L, lam, t, K, m64, n64, J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, 1)
    mud, nud = to_dev(mu), to_dev(nu)
    rec = torch.empty(gs.ckpt_floats(plan, J, gs.GS_RECORD_ALL), device="cuda")
    gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=gs.GS_RECORD_ALL, ckpt=rec)
    gmu = torch.empty(n, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, gs.GS_RECORD_ALL, rec, [1.0], grad_mu=gmu)
    got = to_host(gmu)[coords]
    full = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J)["dmu"][:, 0]
    ratios = {fl: float(np.max(np.abs(got - fd) / np.maximum(np.abs(fd), fl * np.abs(full[m64 > 0]).max())))
              for fl in (1e-3, 1e-2)}
    print(f"worst coordinate error against central differences / max(|fd_i|, floor ||g||_inf): "
          f"1e-3 floor {ratios[1e-3]:.2e}, 1e-2 floor {ratios[1e-2]:.2e}")
    assert ratios[1e-3] <= 1e-4, ratios
    assert gt[0] == pytest.approx(fdt[0], rel=1e-4)


@pytest.mark.parametrize("ce", [5, -1])
def test_autograd_function(gs, clusters, ce):
    """Through torch.autograd, with checkpoints every 5 iterations and with records (-1)."""
    n, labels, arrs, L = clusters
    B, K, J = 2, 20, 10
    rng = np.random.default_rng(77)
    mu, nu = _grad_case(n, labels, B, rng)
    lam = lam_hat_of(L)
    t0 = 1.5
    ref = osk.sinkhorn_grad(L, lam, t0, K, mu.astype(np.float64), nu.astype(np.float64), J)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    mud = to_dev(mu).requires_grad_(True)
    nud = to_dev(nu).requires_grad_(True)
    tt = torch.tensor(t0, dtype=torch.float64, requires_grad=True)
    D = gs.geodesic_sinkhorn_distance(mud.view(-1), nud.view(-1), tt, plan, lam, J, ce)
    D.sum().backward()
    s = mu > 0
    got = to_host(mud.grad).reshape(n, B)
    assert np.linalg.norm(got[s] - ref["dmu"][s]) / np.linalg.norm(ref["dmu"][s]) <= 1e-4
    assert tt.grad.item() == pytest.approx(ref["dt"].sum(), rel=1e-4)


@pytest.mark.parametrize("t_device,t_dtype", [("cuda", torch.float32), ("cpu", torch.float32),
                                              ("cuda", torch.float64)])
def test_autograd_time_gradient_keeps_t_device_and_dtype(gs, clusters, t_device, t_dtype):
    """t given as a device or float32 tensor: its gradient comes back on t's own
    device with t's dtype and shape (autograd rejects anything else)."""
    n, labels, arrs, L = clusters
    B, K, J, t0 = 2, 20, 6, 1.5
    rng = np.random.default_rng(78)
    mu, nu = _grad_case(n, labels, B, rng)
    lam = lam_hat_of(L)
    ref = osk.sinkhorn_grad(L, lam, t0, K, mu.astype(np.float64), nu.astype(np.float64), J)
    plan = gs.Plan(gs.gs_graph_from_csr(n, *arrs), K, B)
    tt = torch.tensor(t0, dtype=t_dtype, device=t_device, requires_grad=True)
    D = gs.geodesic_sinkhorn_distance(to_dev(mu).view(-1), to_dev(nu).view(-1), tt, plan, lam, J)
    D.sum().backward()
    assert tt.grad.device == tt.device and tt.grad.dtype == t_dtype and tt.grad.shape == tt.shape
    assert tt.grad.item() == pytest.approx(ref["dt"].sum(), rel=1e-4)


@pytest.mark.parametrize("K", [1, 2, 3])
@pytest.mark.parametrize("ce", [2, -1])
def test_smallest_degrees_forward_and_backward(gs, clusters, K, ce):
    """K = 1 (the first step is also the last: scaling epilogue and record
    store on it), K = 2 and 3 (one flush before the last step), forward and
    reverse sweep (the dual form on those schedules) against the oracle.
    At t = 0.3 with dense positive histograms every denominator stays above
    the floor (asserted), so both sides take the same branches."""
    n, labels, arrs, L = clusters
    B, t, J = 3, 0.3, 6
    rng = np.random.default_rng(K * 10 + ce)
    mu = synth.random_dense_like(n, B, rng, positive=True)
    nu = synth.random_dense_like(n, B, rng, positive=True)
    mu /= mu.sum(axis=0)
    nu /= nu.sum(axis=0)
    gd = np.array([1.0, -0.5, 2.0])
    lam = lam_hat_of(L)
    ref = osk.sinkhorn_grad(L, lam, t, K, mu.astype(np.float64), nu.astype(np.float64), J, g=gd)
    g = gs.gs_graph_from_csr(n, *arrs)
    plan = gs.Plan(g, K, B)
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device="cuda")
    mud, nud = to_dev(mu), to_dev(nu)
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=ce, ckpt=ckpt, want_floors=True)
    assert out["n_floored"] == 0
    assert (np.abs(out["dist"] - ref["D"]) <= 1e-5 * np.maximum(np.abs(ref["D"]), 4 * t)).all(), (out["dist"], ref["D"])
    gmu = torch.empty(n * B, device="cuda")
    gnu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ckpt, gd, grad_mu=gmu, grad_nu=gnu)
    for got, want in ((to_host(gmu).reshape(n, B), ref["dmu"]), (to_host(gnu).reshape(n, B), ref["dnu"])):
        for b in range(B):
            rel = np.linalg.norm(got[:, b] - want[:, b]) / np.linalg.norm(want[:, b])
            assert rel <= 1e-4, (K, b, rel)
    np.testing.assert_allclose(gt, ref["dt"], rtol=1e-4)

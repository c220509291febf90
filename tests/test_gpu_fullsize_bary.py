"""The barycenter workload at full size, in the benchmark's launch shape.

n = 200k (30 clusters x 6667 in R^50, k = 15), m = 64 inputs with log-uniform
supports of 1k-50k nodes and Dirichlet(0.5) weights, alpha = 1/64, K = 40,
t = 2, the autotuned 64-column plan.  The oracle cannot run the whole
iteration at this size in seconds, but one iteration from w = 1 has a
per-node closed form it can evaluate on sampled nodes:
  p_K 1 = p_K(0) 1 (L 1 = 0), so d = p_K(0) and v_i = mu_i / p_K(0);
  q_i = floor(p_K v_i) with (p_K mu_i)_j = (p_K e_j) . mu_i (p_K symmetric);
  p_j = exp(sum_i alpha_i ln q_ij).
The oracle applies p_K to Diracs at 16 sampled nodes on the library's
exported graph with the same lambda_hat.  Tolerance: the barycenter bar
||p - p_ref||_1 <= 1e-6 read per node, |p_j - p_ref_j| <= 1e-6 p_ref_j (which,
held at every node, gives the L1 bound for a barycenter of mass ~1).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import heat
from gpu_common import csr_laplacian, need_gpu

pytestmark = pytest.mark.gpu


def test_barycenter_first_iteration_on_sampled_nodes():
    need_gpu()
    import paper_2211_00805_amd as gs
    X, _ = synth.clusters_on_curve(30, 6667, dim=50, sigma=0.1, workload=3)
    g = gs.gs_graph_from_points(X, 15)
    assert g.n_components == 1
    lam = gs.gs_lambda_max(g, iters=60, seed=3, safety=1.01)
    n, m, K, t, phi = g.n, 64, 40, 2.0, 1e-30
    H, _ = synth.loguniform_support_histograms(n, m, 1000, 50000, 0.5, np.random.default_rng(synth.seed_for(3, 2)))
    plan = gs.Plan(g, K, m, flags=gs.GS_PLAN_AUTOTUNE)
    alpha = np.full(m, 1.0 / m)
    bary = torch.empty(n, device="cuda")
    gs.gs_barycenter(plan, lam, t, torch.from_numpy(H).cuda(), alpha, 1, bary)
    p_gpu = bary.cpu().numpy().astype(np.float64)

    rp, col, w, _ = g.export()
    L = csr_laplacian(n, (rp, col, w))
    rng = np.random.default_rng(29)
    nodes = rng.choice(n, 16, replace=False)
    E = np.zeros((n, len(nodes)))
    E[nodes, np.arange(len(nodes))] = 1.0
    rows = heat.heat_apply(L, lam, t, K, E)               # column s = p_K e_j = row j of p_K
    b = heat.cheb_coeffs(t, K)
    p0 = b[0] / 2 + sum((-1) ** k * b[k] for k in range(1, K + 1))
    H64 = H.astype(np.float64)
    v = H64 / p0
    q = np.maximum(rows.T @ v, phi)                        # (16, m): q_ij
    ref = np.exp(np.log(q) @ alpha)                        # p_j = prod_i q_ij^alpha_i
    rel = np.abs(p_gpu[nodes] - ref) / ref
    print("max relative error", rel.max(), "plan", plan.describe())
    assert np.all(rel <= 1e-6), rel
    assert np.all(np.isfinite(p_gpu)) and np.all(p_gpu > 0)

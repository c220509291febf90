"""Full-size checks on the 1M-node kNN workload, in the benchmark's launch shape.

The oracle cannot build this graph (brute-force kNN over 1M points in R^100),
so the checks use what it can compute one node at a time and properties that
hold at any size:
  * sampled nodes: exact k nearest neighbours by brute force (float64), every
    directed neighbour present in the library's row, Gaussian weights with a
    single median m (ln w = -d^2 / m^2 on every sampled edge);
  * heat application in the tuned 32-column shape: mass 1^T p_K x = p_K(0) 1^T x
    (L 1 = 0) and symmetry <z, p_K x> = <p_K z, x>, both to float32 rounding;
  * Algorithm 1 + reverse sweep: the column marginal a w p_K(a v) equals a nu
    exactly after a w-update, and the gradient agrees with central differences
    of the GPU forward along a random direction of the supports;
  * Algorithm 1 in the benchmark's tuned 32-column launch for 5 iterations:
    two sampled columns against the float64 oracle run on the library's
    exported graph with the same lambda_hat.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import graph as ograph
from oracle import heat
from oracle import spectrum
from gpu_common import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_2211_00805_amd", "tune_cache.json")


@pytest.fixture(scope="module")
def big():
    need_gpu()
    import paper_2211_00805_amd as gs
    X, labels = synth.clusters_on_surface((10, 5), 20000, 100, 0.1, workload=5)
    g = gs.gs_graph_from_points(X, 10)
    lam = gs.gs_lambda_max(g, iters=60, seed=5, safety=1.01)
    return gs, X, g, lam


def _knn_of(X64, norms, i, k):
    """k nearest other points of point i (float64 Gram distances, ties by id)."""
    d2 = norms + norms[i] - 2.0 * (X64 @ X64[i])
    d2[i] = np.inf
    cand = np.argpartition(d2, k + 4)[:k + 4]
    return set(cand[np.lexsort((cand, d2[cand]))][:k].tolist())


def test_sampled_rows_are_exact_knn_unions(big):
    gs, X, g, lam = big
    rp, col, w, deg = g.export()
    X64 = X.astype(np.float64)
    norms = np.einsum("ij,ij->i", X64, X64)
    rng = np.random.default_rng(17)
    k = 10
    logs = []
    for i in rng.choice(g.n, size=12, replace=False):
        nn = _knn_of(X64, norms, i, k)
        row = col[rp[i]:rp[i + 1]]
        assert nn <= set(row.tolist()), i
        # every other entry j of the row has i among its own k nearest
        for j in set(row.tolist()) - nn:
            assert i in _knn_of(X64, norms, j, k), (i, j)
        ew = w[rp[i]:rp[i + 1]].astype(np.float64)
        logs.append(np.log(ew) / ograph.pair_sqdist(X, np.full(len(row), i), row))
    r = np.concatenate(logs)
    np.testing.assert_allclose(r, -1.0 / g.median ** 2, rtol=2e-6)
    assert g.n_components == 1


def test_lambda_hat_brackets_lambda_max(big):
    """The library's lambda_hat (Lanczos) lies between lambda_max of the exported
    graph's Laplacian (ARPACK, float64) and the edge bound max_E (d_i + d_j):
    the Chebyshev expansion needs the spectrum inside [0, lambda_hat]."""
    gs, X, g, lam = big
    rp, col, w, _ = g.export()
    A = ograph.csr_from_arrays(g.n, rp, col, w.astype(np.float64))
    lmax = spectrum.lambda_max(ograph.laplacian(A))
    eb = spectrum.edge_bound(A)
    print(f"n={g.n}: lambda_max {lmax:.6f} <= lambda_hat {lam:.6f} <= edge bound {eb:.6f}")
    assert lmax * (1 + 1e-9) <= lam <= eb * (1 + 1e-6)


def test_heat_apply_mass_and_symmetry_in_benchmark_shape(big):
    gs, X, g, lam = big
    n, K, t, B = g.n, 50, 2.0, 32
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE)
    rng = np.random.default_rng(3)
    x = synth.random_dense_like(n, B, rng, positive=True)
    z = synth.random_dense_like(n, B, rng)
    Yx = torch.empty(n * B, device="cuda")
    Yz = torch.empty(n * B, device="cuda")
    gs.gs_heat_apply(plan, lam, t, to_dev(x), Yx)
    gs.gs_heat_apply(plan, lam, t, to_dev(z), Yz)
    px = to_host(Yx).reshape(n, B)
    pz = to_host(Yz).reshape(n, B)
    b = heat.cheb_coeffs(t, K)
    p0 = 0.5 * b[0] + np.sum(b[1:] * (-1.0) ** np.arange(1, K + 1))
    np.testing.assert_allclose(px.sum(axis=0), p0 * x.astype(np.float64).sum(axis=0), rtol=1e-4)
    lhs = np.sum(z.astype(np.float64) * px, axis=0)
    rhs = np.sum(pz * x.astype(np.float64), axis=0)
    scale = np.sqrt(np.sum(z.astype(np.float64) ** 2, axis=0) * np.sum(px ** 2, axis=0))
    assert np.all(np.abs(lhs - rhs) <= 1e-5 * scale)
    assert px.min() >= -heat.tail_bound(t, K) * np.abs(x).max()


def test_sinkhorn_gradient_matches_directional_differences(big):
    gs, X, g, lam = big
    n, K, t, J, ce, B = g.n, 50, 2.0, 20, 10, 32
    m = 2 * B
    sizes = synth.loguniform_support_sizes(n, m, 5000, 200000, 77)
    H = np.stack([synth.histogram_on_random_support(n, int(s), 1.0, 770 + i) for i, s in enumerate(sizes)], axis=1)
    mu, nu = H[:, :B].copy(), H[:, B:].copy()
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE)
    mud, nud = to_dev(mu), to_dev(nu)
    ckpt = torch.empty(gs.n_checkpoints(J, ce) * n * B, device="cuda")
    v = torch.empty(n * B, device="cuda")
    w = torch.empty(n * B, device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mud, nud, J, ckpt_every=ce, ckpt=ckpt, v=v, w=w, want_floors=True)
    assert np.all(np.isfinite(out["dist"])) and out["n_floored"] == 0
    # column marginal a w p_K(a v) = nu after the w-update (a = 1)
    pv = torch.empty(n * B, device="cuda")
    plan1 = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE)
    gs.gs_heat_apply(plan1, lam, t, v, pv)
    colm = to_host(w) * to_host(pv)
    np.testing.assert_allclose(colm.reshape(n, B).sum(axis=0), nu.astype(np.float64).sum(axis=0), rtol=1e-5)
    gd = np.ones(B)
    gmu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mud, nud, J, ce, ckpt, gd, grad_mu=gmu)
    # direction on the supports, relative step 1e-3
    rng = np.random.default_rng(5)
    dirn = np.where(mu > 0, rng.uniform(-1, 1, size=mu.shape) * mu, 0.0)
    h = 1e-3
    Dp = gs.gs_sinkhorn(plan, lam, t, to_dev(mu + h * dirn), nud, J)["dist"]
    Dm = gs.gs_sinkhorn(plan, lam, t, to_dev(mu - h * dirn), nud, J)["dist"]
    fd = (Dp - Dm) / (2 * h)
    an = np.sum(to_host(gmu).reshape(n, B) * dirn, axis=0)
    np.testing.assert_allclose(an, fd, rtol=2e-3, atol=1e-3 * np.abs(an).max())
    ht = 1e-3
    ftd = (gs.gs_sinkhorn(plan, lam, t + ht, mud, nud, J)["dist"]
           - gs.gs_sinkhorn(plan, lam, t - ht, mud, nud, J)["dist"]) / (2 * ht)
    np.testing.assert_allclose(gt, ftd, rtol=2e-3, atol=1e-3 * np.abs(gt).max())


def test_sinkhorn_columns_match_oracle_at_full_size(big):
    """The benchmark's launch configuration (tuned 32-column plan, K = 50, t = 2)
    for J = 5 iterations, two sampled columns against the float64 oracle run on
    the library's exported graph (float32 weights) with the same lambda_hat."""
    gs, X, g, lam = big
    n, K, t, J, B = g.n, 50, 2.0, 5, 32
    sizes = synth.loguniform_support_sizes(n, 2 * B, 5000, 200000, 91)
    H = np.stack([synth.histogram_on_random_support(n, int(s), 1.0, 910 + i) for i, s in enumerate(sizes)], axis=1)
    mu, nu = H[:, :B].copy(), H[:, B:].copy()
    plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE)
    out = gs.gs_sinkhorn(plan, lam, t, to_dev(mu), to_dev(nu), J)
    rp, col, w, _ = g.export()
    L = ograph.laplacian(ograph.csr_from_arrays(n, rp, col, w.astype(np.float64)))
    cols = [0, 17]
    from oracle import sinkhorn as osk
    ref = osk.sinkhorn(L, lam, t, K, mu[:, cols].astype(np.float64), nu[:, cols].astype(np.float64), J,
                       marginals=False)["D"]
    got = out["dist"][cols]
    assert np.all(np.abs(got - ref) <= 1e-5 * np.maximum(np.abs(ref), 4 * t)), (got, ref)


def test_gradient_accumulation_at_full_size():
    """The benchmark's per-histogram accumulation at its size (n = 1M, 32
    columns into 256 x n, two calls): sampled nodes and both ends, bitwise
    equal to the float32 sums in column order; rows of G that no column
    names stay zero."""
    need_gpu()
    import paper_2211_00805_amd as gs
    n, B, m = 1_000_000, 32, 256
    rng = np.random.default_rng(23)
    src = rng.standard_normal((n, B)).astype(np.float32)
    cols = rng.integers(0, m, B).astype(np.int32)
    cols[5] = cols[6] = cols[7]                       # a histogram in three pairs of the batch
    G = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    dcols = torch.from_numpy(cols).cuda()
    gs.gs_accumulate_columns(to_dev(src), dcols, G)
    gs.gs_accumulate_columns(to_dev(src[:, ::-1].copy()), dcols, G)
    nodes = np.concatenate([[0, 1, 255, 256, n - 1], rng.choice(n, 4000, replace=False)])
    ref = np.zeros((m, len(nodes)), dtype=np.float32)
    for s in (src, src[:, ::-1]):
        for b in range(B):
            ref[cols[b]] = (ref[cols[b]] + s[nodes, b]).astype(np.float32)
    got = G[:, torch.from_numpy(nodes).cuda()].cpu().numpy()
    assert np.array_equal(got, ref)
    untouched = np.setdiff1d(np.arange(m), cols)
    assert float(G[torch.from_numpy(untouched).cuda()].abs().max()) == 0.0

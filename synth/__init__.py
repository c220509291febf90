"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module only draws random data: point clouds on manifolds, histograms on
random node subsets, and plain random sparse graphs used as operator inputs.
It holds none of the method's arithmetic (no affinity kernel, no Laplacian,
no Chebyshev or Sinkhorn step), so importing it from both sides shares no
part of what is being checked.

Seeds follow one convention: for workload number c, ``1000*c + 0`` draws the
points, ``1000*c + 1`` draws lifts and spline knots, ``1000*c + 2`` draws
histograms.  Every array can be fingerprinted with :func:`sha256`.
"""
from __future__ import annotations

import hashlib

import numpy as np
from scipy.interpolate import CubicSpline, RectBivariateSpline

__all__ = [
    "sha256",
    "seed_for",
    "swiss_roll",
    "gaussians_on_swiss_roll",
    "clusters_on_curve",
    "clusters_on_surface",
    "uniform_on_random_nodes",
    "dirichlet_on_nodes",
    "cluster_block_pair",
    "loguniform_support_histograms",
    "random_local_graph",
    "cycle_graph",
    "torus_graph",
    "complete_graph",
    "random_dense_like",
    "loguniform_support_sizes",
    "histogram_on_random_support",
    "curve_pair_workload",
    "barycenter_workload",
    "gradient_pairs",
    "local_graph_1m",
    "loguniform_pair_batch",
]


def sha256(a: np.ndarray) -> str:
    """Hex digest of an array's dtype, shape and bytes (for run logs)."""
    a = np.ascontiguousarray(a)
    h = hashlib.sha256()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(a.tobytes())
    return h.hexdigest()


def seed_for(workload: int, stream: int) -> int:
    """Seed for stream 0 (points), 1 (lift/knots) or 2 (histograms)."""
    return 1000 * int(workload) + int(stream)


# ----------------------------------------------------------------------------
# point clouds
# ----------------------------------------------------------------------------

def swiss_roll(n: int = 2000, dim: int = 10, noise: float = 0.05, workload: int = 1) -> np.ndarray:
    """2-D Swiss roll in R^3 lifted to R^dim by a random orthonormal map, plus noise.

    u ~ 1.5*pi*(1 + 2U), h ~ 21U, point (u cos u, h, u sin u); the lift is the Q
    factor of a Gaussian dim x 3 matrix; isotropic N(0, noise^2) noise in R^dim.
    Returns float32 (n, dim).
    """
    rng = np.random.default_rng(seed_for(workload, 0))
    u = 1.5 * np.pi * (1.0 + 2.0 * rng.random(n))
    h = 21.0 * rng.random(n)
    roll = np.stack([u * np.cos(u), h, u * np.sin(u)], axis=1)
    lift_rng = np.random.default_rng(seed_for(workload, 1))
    q, _ = np.linalg.qr(lift_rng.standard_normal((dim, 3)))
    pts = roll @ q.T + noise * rng.standard_normal((n, dim))
    return pts.astype(np.float32)


def _roll_arclength(u: np.ndarray) -> np.ndarray:
    """Arc length of the spiral (u cos u, u sin u) from u = 0."""
    return 0.5 * (u * np.sqrt(1.0 + u * u) + np.arcsinh(u))


def _roll_param_of_arclength(s: np.ndarray) -> np.ndarray:
    """Inverse of _roll_arclength by Newton's method (s > 0)."""
    u = np.sqrt(2.0 * np.maximum(s, 1e-12))
    for _ in range(60):
        u = np.maximum(u - (_roll_arclength(u) - s) / np.sqrt(1.0 + u * u), 1e-9)
    return u


def gaussians_on_swiss_roll(n_dists: int = 15, per_dist: int = 10000, dim: int = 10, sigma: float = 2.5,
                            noise: float = 0.0, workload: int = 6) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Samples of Gaussian distributions on a Swiss roll, rotated into R^dim.

    Intrinsic coordinates are (arc length s along the spiral u in
    [1.5 pi, 4.5 pi], height h in [0, 21]); the roll is a developable surface,
    so geodesic distances are Euclidean in (s, h).  Means are uniform in the
    strip shrunk by 2 sigma on each side; each distribution draws `per_dist`
    points mean + N(0, sigma^2 I_2) in (s, h), mapped to (u cos u, h, u sin u)
    and rotated into R^dim by the Q factor of a Gaussian dim x 3 matrix, plus
    optional isotropic noise.  Points are emitted distribution by
    distribution.  Returns (points float32 (n_dists*per_dist, dim),
    labels int32, means float64 (n_dists, 2) in (s, h)).
    """
    rng = np.random.default_rng(seed_for(workload, 0))
    s_lo, s_hi = _roll_arclength(np.array([1.5 * np.pi, 4.5 * np.pi]))
    lo = np.array([s_lo + 2 * sigma, 2 * sigma])
    hi = np.array([s_hi - 2 * sigma, 21.0 - 2 * sigma])
    means = lo + (hi - lo) * rng.random((n_dists, 2))
    sh = np.repeat(means, per_dist, axis=0) + sigma * rng.standard_normal((n_dists * per_dist, 2))
    u = _roll_param_of_arclength(sh[:, 0])
    roll = np.stack([u * np.cos(u), sh[:, 1], u * np.sin(u)], axis=1)
    lift_rng = np.random.default_rng(seed_for(workload, 1))
    q, _ = np.linalg.qr(lift_rng.standard_normal((dim, 3)))
    pts = roll @ q.T
    if noise > 0:
        pts = pts + noise * rng.standard_normal(pts.shape)
    labels = np.repeat(np.arange(n_dists, dtype=np.int32), per_dist)
    return pts.astype(np.float32), labels, means


def _scale_to_spacing(centers: np.ndarray, spacing: float, pairs: np.ndarray) -> np.ndarray:
    """Scale centers about their mean so the mean distance over `pairs` is `spacing`."""
    c0 = centers - centers.mean(axis=0, keepdims=True)
    gaps = np.linalg.norm(c0[pairs[:, 0]] - c0[pairs[:, 1]], axis=1)
    return c0 * (spacing / gaps.mean())


def clusters_on_curve(n_clusters: int, per_cluster: int, dim: int = 50, sigma: float = 0.1,
                      n_knots: int = 10, spacing: float = 0.35, workload: int = 2,
                      shuffle_within: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian clusters placed along a random smooth curve in R^dim.

    The curve is a natural cubic spline through `n_knots` standard-normal knots;
    the cluster centers sit at `n_clusters` equally spaced curve parameters and
    are scaled so that adjacent centers are `spacing` apart on average.  Points
    are center + N(0, sigma^2 I), emitted cluster by cluster (node ids of one
    cluster are contiguous, their order within the cluster is random).
    Returns (points float32 (n, dim), cluster label int32 (n,)).
    """
    krng = np.random.default_rng(seed_for(workload, 1))
    knots = krng.standard_normal((n_knots, dim))
    spline = CubicSpline(np.linspace(0.0, 1.0, n_knots), knots, bc_type="natural", axis=0)
    centers = spline(np.linspace(0.0, 1.0, n_clusters))
    pairs = np.stack([np.arange(n_clusters - 1), np.arange(1, n_clusters)], axis=1)
    centers = _scale_to_spacing(centers, spacing, pairs)
    rng = np.random.default_rng(seed_for(workload, 0))
    pts = np.repeat(centers, per_cluster, axis=0) + sigma * rng.standard_normal((n_clusters * per_cluster, dim))
    labels = np.repeat(np.arange(n_clusters, dtype=np.int32), per_cluster)
    if shuffle_within:
        for c in range(n_clusters):
            sl = slice(c * per_cluster, (c + 1) * per_cluster)
            pts[sl] = pts[sl][rng.permutation(per_cluster)]
    return pts.astype(np.float32), labels


def clusters_on_surface(grid: tuple[int, int] = (10, 5), per_cluster: int = 20000, dim: int = 100,
                        sigma: float = 0.1, knot_grid: int = 4, spacing: float = 0.35,
                        workload: int = 5) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian clusters placed on a random smooth 2-D surface in R^dim.

    The surface is a tensor-product cubic spline through a `knot_grid` x
    `knot_grid` grid of standard-normal knots (one spline per coordinate);
    centers sit on a grid[0] x grid[1] parameter grid and are scaled so that
    grid-adjacent centers are `spacing` apart on average.
    Returns (points float32 (n, dim), cluster label int32 (n,)).
    """
    krng = np.random.default_rng(seed_for(workload, 1))
    kg = np.linspace(0.0, 1.0, knot_grid)
    knots = krng.standard_normal((knot_grid, knot_grid, dim))
    gu = np.linspace(0.0, 1.0, grid[0])
    gv = np.linspace(0.0, 1.0, grid[1])
    centers = np.empty((grid[0], grid[1], dim))
    for c in range(dim):
        sp = RectBivariateSpline(kg, kg, knots[:, :, c], kx=3, ky=3)
        centers[:, :, c] = sp(gu, gv)
    centers = centers.reshape(-1, dim)
    idx = np.arange(grid[0] * grid[1]).reshape(grid)
    pairs = np.concatenate([
        np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1),
        np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)])
    centers = _scale_to_spacing(centers, spacing, pairs)
    rng = np.random.default_rng(seed_for(workload, 0))
    ncl = centers.shape[0]
    pts = np.empty((ncl * per_cluster, dim), dtype=np.float32)
    for c in range(ncl):  # chunked to bound the float64 temporaries at n = 1M, dim = 100
        blk = centers[c] + sigma * rng.standard_normal((per_cluster, dim))
        pts[c * per_cluster:(c + 1) * per_cluster] = blk.astype(np.float32)
    labels = np.repeat(np.arange(ncl, dtype=np.int32), per_cluster)
    return pts, labels


# ----------------------------------------------------------------------------
# histograms (dense length-n float32 vectors, zero off the support)
# ----------------------------------------------------------------------------

def uniform_on_random_nodes(n: int, size: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform weights 1/size on `size` nodes drawn without replacement."""
    h = np.zeros(n, dtype=np.float64)
    h[rng.choice(n, size=size, replace=False)] = 1.0 / size
    return h.astype(np.float32)


def dirichlet_on_nodes(n: int, nodes: np.ndarray, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Dirichlet(alpha) weights on the given node ids (float64 draw, float32 out)."""
    h = np.zeros(n, dtype=np.float64)
    h[nodes] = rng.dirichlet(np.full(len(nodes), alpha))
    return h.astype(np.float32)


def cluster_block_pair(labels: np.ndarray, first: int, width: int, alpha: float,
                       rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Two Dirichlet(alpha) histograms on adjacent blocks of `width` clusters.

    mu lives on clusters [first, first+width), nu on [first+width, first+2*width).
    """
    n = labels.shape[0]
    a = np.nonzero((labels >= first) & (labels < first + width))[0]
    b = np.nonzero((labels >= first + width) & (labels < first + 2 * width))[0]
    return dirichlet_on_nodes(n, a, alpha, rng), dirichlet_on_nodes(n, b, alpha, rng)


def loguniform_support_histograms(n: int, m: int, lo: int, hi: int, alpha: float,
                                  rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """m histograms with support sizes floor(exp(U[ln lo, ln hi])) on random nodes.

    Returns (H float32 (n, m) node-major, sizes int64 (m,)).
    """
    sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=m))).astype(np.int64)
    sizes = np.clip(sizes, 1, n)
    H = np.zeros((n, m), dtype=np.float32)
    for i, s in enumerate(sizes):
        nodes = rng.choice(n, size=int(s), replace=False)
        H[:, i] = dirichlet_on_nodes(n, nodes, alpha, rng)
    return H, sizes


def loguniform_support_sizes(n: int, m: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Support sizes floor(exp(U[ln lo, ln hi])) of m histograms, clipped to [1, n]."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=m))).astype(np.int64)
    return np.clip(sizes, 1, n)


def histogram_on_random_support(n: int, size: int, alpha: float, seed: int) -> np.ndarray:
    """One Dirichlet(alpha) histogram on `size` nodes drawn without replacement (own seed)."""
    rng = np.random.default_rng(seed)
    return dirichlet_on_nodes(n, rng.choice(n, size=int(size), replace=False), alpha, rng)


def random_dense_like(n: int, B: int, rng: np.random.Generator, positive: bool = False) -> np.ndarray:
    """Dense float32 (n, B) test signal: N(0,1), or U(0.05, 1) when positive."""
    if positive:
        return rng.uniform(0.05, 1.0, size=(n, B)).astype(np.float32)
    return rng.standard_normal((n, B)).astype(np.float32)


# ----------------------------------------------------------------------------
# plain graphs as CSR arrays (int32 rowptr/col, float32 weights)
# ----------------------------------------------------------------------------

def _csr_from_undirected(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray):
    """CSR (rowptr, col, val) of the symmetric matrix with entries (i,j)=(j,i)=w."""
    r = np.concatenate([i, j])
    c = np.concatenate([j, i])
    v = np.concatenate([w, w])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), c.astype(np.int32), v.astype(np.float32)


def random_local_graph(n: int, k: int, window: int, rng: np.random.Generator,
                       wlo: float = 0.05, whi: float = 1.0, hubs: int = 0, hub_degree: int = 0):
    """Random symmetric sparse graph with kNN-like size and locality.

    Every node i draws k partners uniformly from the `window` ids on either side
    of i (wrapping around), self pairs dropped; the undirected edge set is the
    union of the draws, each edge gets a U(wlo, whi) weight.  Degree profile and
    nonzeros per row resemble a symmetrised kNN graph, gathers stay within a
    band.  Optionally `hubs` random nodes are linked to `hub_degree` random
    nodes each (the high-degree rows of kNN graphs in high dimension).
    Returns CSR (rowptr int32, col int32, w float32).
    """
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    off = rng.integers(1, window + 1, size=n * k) * rng.choice(np.array([-1, 1]), size=n * k)
    dst = (src + off) % n
    if hubs:
        hub_ids = rng.choice(n, size=hubs, replace=False)
        src = np.concatenate([src, np.repeat(hub_ids, hub_degree)])
        dst = np.concatenate([dst, rng.integers(0, n, size=hubs * hub_degree)])
    a = np.minimum(src, dst)
    b = np.maximum(src, dst)
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    i, j = key // n, key % n
    w = rng.uniform(wlo, whi, size=key.shape[0])
    return _csr_from_undirected(n, i, j, w)


def cycle_graph(n: int):
    """Unit-weight cycle C_n as CSR."""
    i = np.arange(n, dtype=np.int64)
    j = (i + 1) % n
    return _csr_from_undirected(n, i, j, np.ones(n))


def torus_graph(n1: int, n2: int):
    """Unit-weight 2-D torus C_n1 x C_n2 (node id = a*n2 + b) as CSR."""
    a, b = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    u = (a * n2 + b).ravel()
    right = (a * n2 + (b + 1) % n2).ravel()
    down = (((a + 1) % n1) * n2 + b).ravel()
    i = np.concatenate([u, u])
    j = np.concatenate([right, down])
    return _csr_from_undirected(n1 * n2, i, j, np.ones(i.shape[0]))


def complete_graph(n: int):
    """Unit-weight complete graph K_n as CSR."""
    i, j = np.triu_indices(n, 1)
    return _csr_from_undirected(n, i, j, np.ones(i.shape[0]))


# ----------------------------------------------------------------------------
# the paper-shaped workloads (points or graph plus histograms), one recipe each
# ----------------------------------------------------------------------------

def curve_pair_workload(per_cluster: int = 5000, n_clusters: int = 20):
    """Plain forward: clusters on a curve in R^50 (workload 2) and one histogram pair.

    mu = Dirichlet(1) on clusters 0-3, nu = Dirichlet(1) on clusters 4-7.
    Returns (X float32 (n, 50), labels, mu float32 (n,), nu float32 (n,)).
    """
    X, labels = clusters_on_curve(n_clusters, per_cluster, dim=50, sigma=0.1, workload=2)
    mu, nu = cluster_block_pair(labels, 0, 4, 1.0, np.random.default_rng(seed_for(2, 2)))
    return X, labels, mu, nu


def barycenter_workload(per_cluster: int = 6667, lo: int = 1000, hi: int = 50000, m: int = 64):
    """Barycenter: 30 clusters on a curve in R^50 (workload 3) and m input histograms.

    Supports of log-uniform size in [lo, hi] on random nodes, Dirichlet(0.5).
    Returns (X float32 (n, 50), labels, H float32 (n, m)).
    """
    X, labels = clusters_on_curve(30, per_cluster, dim=50, sigma=0.1, workload=3)
    H, _ = loguniform_support_histograms(X.shape[0], m, lo, hi, 0.5, np.random.default_rng(seed_for(3, 2)))
    return X, labels, H


def gradient_pairs(labels: np.ndarray, B: int = 32, width: int = 3):
    """Differentiation: B Dirichlet(1) pairs on adjacent blocks of `width` clusters.

    Each pair starts at a random cluster (seed of workload 4); mu covers
    clusters [s, s+width), nu the next `width`.  Returns (mu, nu) float32 (n, B).
    """
    rng = np.random.default_rng(seed_for(4, 2))
    ncl = int(labels.max()) + 1
    pairs = [cluster_block_pair(labels, int(rng.integers(0, ncl - 2 * width)), width, 1.0, rng) for _ in range(B)]
    return np.stack([p[0] for p in pairs], axis=1), np.stack([p[1] for p in pairs], axis=1)


def local_graph_1m(n: int = 1_000_000):
    """A 1M-node random local graph with the 1M kNN workload's size (workload 10).

    k = 9 partners per node within a window of 20,000 ids plus 200 hub nodes of
    1000 extra random partners each: about 18.4M nonzeros (the kNN graph has
    18.3M) and rows long enough for the long-row path.  Returns CSR arrays.
    """
    return random_local_graph(n, 9, 20000, np.random.default_rng(seed_for(10, 0)), hubs=200, hub_degree=1000)


def loguniform_pair_batch(n: int, B: int, lo: int, hi: int, workload: int):
    """B histogram pairs with log-uniform support sizes in [lo, hi], Dirichlet(1).

    Histogram i (0..2B-1) has its own seed seed_for(workload, 2) * 1000 + i;
    pair b is (histogram 2b, histogram 2b+1).  Returns (mu, nu) float32 (n, B).
    """
    sizes = loguniform_support_sizes(n, 2 * B, lo, hi, seed_for(workload, 2))
    mu = np.empty((n, B), dtype=np.float32)
    nu = np.empty((n, B), dtype=np.float32)
    for b in range(B):
        mu[:, b] = histogram_on_random_support(n, int(sizes[2 * b]), 1.0, seed_for(workload, 2) * 1000 + 2 * b)
        nu[:, b] = histogram_on_random_support(n, int(sizes[2 * b + 1]), 1.0, seed_for(workload, 2) * 1000 + 2 * b + 1)
    return mu, nu

"""Common kNN affinity graph and combinatorial Laplacian (oracle, float64).

Paper: Sec. "Geodesic Sinkhorn Distances" builds one graph over all datasets
with an affinity kernel; Sec. "Heat Diffusion on a Graph" defines the degree
matrix D_ii = sum_k A_ik and the combinatorial Laplacian L = D - A.

Reading (the paper names no kernel or k): the graph is the union of the
directed k-nearest-neighbour edges (self excluded, equal distances broken
towards the lower node id), with Gaussian weights exp(-d^2 / m^2) where m is
the median of the n*k directed kNN distances.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy.spatial.distance import cdist


def knn_lists(X: np.ndarray, k: int, block: int = 512, rows: tuple[int, int] | None = None):
    """k nearest other points of every point, by Euclidean distance.

    Brute force over row blocks with direct squared differences (cdist).
    Order within a row is by (distance, node id); equal distances go to the
    lower id.  Returns (idx int64 (n, k), d2 float64 (n, k)); with
    rows = (lo, hi) only the points lo..hi-1 are searched (against all n
    points) and the arrays have hi - lo rows, so a large cloud can be split
    over processes.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if not 1 <= k < n:
        raise ValueError("need 1 <= k < n")
    lo, hi = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    if not 0 <= lo <= hi <= n:
        raise ValueError("rows out of range")
    idx = np.empty((hi - lo, k), dtype=np.int64)
    d2 = np.empty((hi - lo, k), dtype=np.float64)
    for r0 in range(lo, hi, block):
        r1 = min(hi, r0 + block)
        D = cdist(X[r0:r1], X, metric="sqeuclidean")
        D[np.arange(r1 - r0), np.arange(r0, r1)] = np.inf  # no self edge
        thresh = np.partition(D, k - 1, axis=1)[:, k - 1]
        for r in range(r1 - r0):
            cand = np.nonzero(D[r] <= thresh[r])[0]          # ascending ids
            order = np.lexsort((cand, D[r, cand]))[:k]       # by distance, then id
            idx[r0 - lo + r] = cand[order]
            d2[r0 - lo + r] = D[r, cand[order]]
    return idx, d2


def pair_sqdist(X: np.ndarray, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance of point pairs, summed over coordinates."""
    X = np.asarray(X, dtype=np.float64)
    diff = X[i] - X[j]
    return np.einsum("ed,ed->e", diff, diff)


def gaussian_weights(X: np.ndarray, i: np.ndarray, j: np.ndarray, m: float) -> np.ndarray:
    """Affinity exp(-||x_i - x_j||^2 / m^2) of the point pairs (i, j)."""
    return np.exp(-pair_sqdist(X, i, j) / (m * m))


def knn_graph(X: np.ndarray, k: int, knn_idx: np.ndarray | None = None):
    """Symmetrised kNN graph with Gaussian-median weights.

    Returns (A, info): A is a float64 scipy CSR adjacency with sorted column
    ids and no self loops; info holds the directed kNN lists, the median
    distance m and the component count.  knn_idx, when given, is the (n, k)
    result of knn_lists (e.g. assembled from row ranges searched apart).
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    idx = knn_lists(X, k)[0] if knn_idx is None else np.asarray(knn_idx, dtype=np.int64)
    if idx.shape != (n, k):
        raise ValueError("knn_idx must be (n, k)")
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = idx.ravel()
    d_dir = np.sqrt(pair_sqdist(X, src, dst))               # directed kNN distances
    m = float(np.median(d_dir))
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    key = np.unique(lo * n + hi)                           # union of the directed edges
    a, b = key // n, key % n
    w = gaussian_weights(X, a, b, m)
    A = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([a, b]), np.concatenate([b, a]))),
                      shape=(n, n)).tocsr()
    A.sort_indices()
    ncomp, _ = connected_components(A, directed=False)
    info = {"knn_idx": idx, "median": m, "n_components": int(ncomp), "directed_dist": d_dir}
    return A, info


def csr_from_arrays(n: int, rowptr, col, val) -> sp.csr_matrix:
    """float64 scipy CSR from (rowptr, col, val) arrays."""
    A = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col, dtype=np.int64),
                       np.asarray(rowptr, dtype=np.int64)), shape=(n, n))
    A.sort_indices()
    return A


def laplacian(A: sp.spmatrix) -> sp.csr_matrix:
    """Combinatorial Laplacian L = D - A with D_ii = sum_k A_ik."""
    A = sp.csr_matrix(A, dtype=np.float64)
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(deg) - A).tocsr()

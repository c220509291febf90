"""All-pairs distances and nearest-neighbour scores (oracle, float64).

Test infrastructure only.  Paper, Sec. "Nearest-Wasserstein-neighbor
distributions" (Table 1): the distance between two of m distributions is
Algorithm 1's return value for that pair; the task is scored by Spearman and
Pearson correlation of the pairwise distances (i < j) with ground-truth
distances, and by the precision at 5 of each distribution's nearest
neighbours (self excluded).  Correlations are scipy's.  The gradient of the
total of the pairwise distances with respect to each distribution is the sum,
over the pairs that contain it, of the pair's gradient in that argument (chain
rule; a pair (i, i) contributes its gradient in both arguments).
"""
from __future__ import annotations

import numpy as np
from scipy import stats

from .sinkhorn import sinkhorn, sinkhorn_grad


def distance_matrix(L, lam_hat, t, K, H, J, diagonal=False):
    """D[i, j] = D[j, i] = Algorithm 1 (mu = H[:, i], nu = H[:, j]), all pairs at once as columns."""
    H = np.asarray(H, dtype=np.float64)
    m = H.shape[1]
    pairs = [(i, j) for i in range(m) for j in range(i if diagonal else i + 1, m)]
    D = np.zeros((m, m))
    if not pairs:
        return D
    I = np.array([p[0] for p in pairs])
    Jx = np.array([p[1] for p in pairs])
    d = sinkhorn(L, lam_hat, t, K, H[:, I], H[:, Jx], J, marginals=False)["D"]
    D[I, Jx] = d
    D[Jx, I] = d
    return D


def total_gradient(L, lam_hat, t, K, H, J, diagonal=False):
    """Total T = sum of D(H[:, i], H[:, j]) over the pairs i < j (i <= j with the
    diagonal) and its gradient G (n, m) with respect to every column of H
    (reported on each column's support, zero elsewhere), through exactly J
    iterations."""
    H = np.asarray(H, dtype=np.float64)
    n, m = H.shape
    pairs = [(i, j) for i in range(m) for j in range(i if diagonal else i + 1, m)]
    G = np.zeros((n, m))
    if not pairs:
        return 0.0, G
    I = np.array([p[0] for p in pairs])
    Jx = np.array([p[1] for p in pairs])
    out = sinkhorn_grad(L, lam_hat, t, K, H[:, I], H[:, Jx], J)
    for p, (i, j) in enumerate(pairs):
        G[:, i] += out["dmu"][:, p]
        G[:, j] += out["dnu"][:, p]
    return float(np.sum(out["D"])), G


def knn_sets(D, k):
    """Each row's k nearest other indices (ties to the lower index)."""
    m = D.shape[0]
    out = []
    for i in range(m):
        cand = sorted((D[i, j], j) for j in range(m) if j != i)
        out.append({j for _, j in cand[:k]})
    return out


def nn_scores(D, truth, k=5):
    iu = np.triu_indices(D.shape[0], 1)
    d, g = D[iu], truth[iu]
    a, b = knn_sets(D, k), knn_sets(truth, k)
    p = sum(len(x & y) for x, y in zip(a, b)) / (k * D.shape[0])
    return {"spearman": float(stats.spearmanr(d, g).statistic), "pearson": float(stats.pearsonr(d, g).statistic),
            f"p_at_{k}": p}

"""All-pairs Geodesic Sinkhorn distances and nearest-neighbour scores.

Sec. "Nearest-Wasserstein-neighbor distributions" (Table 1): the distances
between m distributions on one graph are Algorithm 1's return value for every
pair; the task is scored by the Spearman and Pearson correlation of the
off-diagonal distances with ground-truth distances, and by the precision at 5
of each distribution's nearest neighbours.

`distance_matrix` runs the pairs i < j through one plan, B pairs per batch
(each batch's columns gathered from H by `gs_gather_columns`, then one
`gs_sinkhorn` call: B right-hand sides per step launch), with
B = `batch` (or the next power of two above P when there are only P < batch
pairs); a short last batch is padded with copies of its first pair, whose
results are dropped.  Widths whose padded row (B rounded up to 4 floats) is a
power of two let each gathered row be read by one group of lanes in one
pass: at n = 150k an odd width such as 35 costs 5x more per launch than 32.
With `grad`, each batch also runs the reverse sweep (`gs_sinkhorn_backward`,
reading the forward's recorded denominators) and `gs_accumulate_columns` adds
its per-pair gradients into the per-histogram gradients of the total of the
computed distances.  The scores are plain definitions over the m x m
matrices.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import (GS_RECORD_ALL, Graph, Plan, ckpt_floats, gs_accumulate_columns, gs_gather_columns, gs_sinkhorn,
                  gs_sinkhorn_backward)


def pair_list(m: int, diagonal: bool = False) -> np.ndarray:
    """Pairs (i, j), i < j (i <= j with the diagonal), row by row."""
    return np.array([(i, j) for i in range(m) for j in range(i if diagonal else i + 1, m)], dtype=np.int64)


def distance_matrix(graph: Graph, lambda_hat: float, t: float, K: int, H: torch.Tensor, iters: int,
                    batch: int = 32, diagonal: bool = False, phi: float = 1e-30, plan: Plan | None = None,
                    plan_flags: int = 0, tune_cache: str | None = None, grad: bool = False):
    """Symmetric m x m matrix of Algorithm 1's distances between the columns of H (n, m).

    D[i, j] = D[j, i] is the distance with mu = H[:, i], nu = H[:, j] (i < j);
    the diagonal holds the self-distances when `diagonal`, else 0.
    With `grad`, returns (D, G): G (m, n) float32 on H's device holds the
    gradient of the total sum_{computed pairs} D_ij with respect to each
    column of H (zero off each column's support), through exactly `iters`
    iterations; the forward records every iteration's denominators
    (2 * iters * n * B floats of device memory).
    """
    if H.dim() != 2 or H.shape[0] != graph.n:
        raise ValueError(f"H must be (n={graph.n}, m), got {tuple(H.shape)}")
    if H.dtype != torch.float32 or H.device.type != "cuda":
        raise TypeError("H must be a float32 device tensor")
    H = H.contiguous()
    m = H.shape[1]
    pairs = pair_list(m, diagonal)
    D = np.zeros((m, m), dtype=np.float64)
    G = torch.zeros((m, graph.n), dtype=torch.float32, device=H.device) if grad else None
    if len(pairs) == 0:
        return (D, G) if grad else D
    B = min(batch, 1 << (len(pairs) - 1).bit_length())
    if plan is None:
        plan = Plan(graph, K, B, flags=plan_flags, tune_cache=tune_cache)
    elif plan.B != B or plan.K != K:
        raise ValueError("plan does not match (K, batch)")
    mu = torch.empty((graph.n, B), dtype=torch.float32, device=H.device)
    nu = torch.empty_like(mu)
    if grad:
        rec = torch.empty(ckpt_floats(plan, iters, GS_RECORD_ALL), dtype=torch.float32, device=H.device)
        gmu = torch.empty((graph.n, B), dtype=torch.float32, device=H.device)
        gnu = torch.empty_like(gmu)
    for s in range(0, len(pairs), B):
        blk = pairs[s:s + B]
        nreal = len(blk)
        if nreal < B:
            blk = np.concatenate([blk, np.repeat(blk[:1], B - nreal, axis=0)])
        gs_gather_columns(H, torch.from_numpy(blk[:, 0].astype(np.int32)).to(H.device), mu)
        gs_gather_columns(H, torch.from_numpy(blk[:, 1].astype(np.int32)).to(H.device), nu)
        if grad:
            d = gs_sinkhorn(plan, lambda_hat, t, mu, nu, iters, phi=phi, ckpt_every=GS_RECORD_ALL,
                            ckpt=rec)["dist"][:nreal]
            weight = np.zeros(B)
            weight[:nreal] = 1.0                 # padding pairs add nothing
            gs_sinkhorn_backward(plan, lambda_hat, t, mu, nu, iters, GS_RECORD_ALL, rec, weight, phi=phi,
                                 grad_mu=gmu, grad_nu=gnu, want_grad_t=False)
            for side, g in ((0, gmu), (1, gnu)):
                cols = np.full(B, -1, dtype=np.int32)
                cols[:nreal] = blk[:nreal, side]
                gs_accumulate_columns(g, torch.from_numpy(cols).to(H.device), G)
        else:
            d = gs_sinkhorn(plan, lambda_hat, t, mu, nu, iters, phi=phi)["dist"][:nreal]
        D[blk[:nreal, 0], blk[:nreal, 1]] = d
        D[blk[:nreal, 1], blk[:nreal, 0]] = d
    return (D, G) if grad else D


def _average_ranks(x: np.ndarray) -> np.ndarray:
    """Ranks 1..N with ties given the mean of their positions."""
    order = np.argsort(x, kind="mergesort")
    xs = x[order]
    ranks = np.empty(len(x), dtype=np.float64)
    i = 0
    while i < len(x):
        j = i
        while j + 1 < len(x) and xs[j + 1] == xs[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return ranks


def _pearson(x: np.ndarray, y: np.ndarray) -> float:
    xc = x - x.mean()
    yc = y - y.mean()
    return float(np.dot(xc, yc) / np.sqrt(np.dot(xc, xc) * np.dot(yc, yc)))


def precision_at_k(D: np.ndarray, truth: np.ndarray, k: int = 5) -> float:
    """Mean over rows of |kNN_D(i) & kNN_truth(i)| / k, self excluded (ties to the lower index)."""
    m = D.shape[0]
    hits = 0
    for i in range(m):
        others = np.array([j for j in range(m) if j != i])
        a = others[np.lexsort((others, D[i, others]))][:k]
        b = others[np.lexsort((others, truth[i, others]))][:k]
        hits += len(set(a.tolist()) & set(b.tolist()))
    return hits / (k * m)


def nn_scores(D: np.ndarray, truth: np.ndarray, k: int = 5) -> dict:
    """Spearman and Pearson correlation over the pairs i < j, and precision at k."""
    iu = np.triu_indices(D.shape[0], 1)
    d, g = np.asarray(D, dtype=np.float64)[iu], np.asarray(truth, dtype=np.float64)[iu]
    return {"spearman": _pearson(_average_ranks(d), _average_ranks(g)), "pearson": _pearson(d, g),
            f"p_at_{k}": precision_at_k(D, truth, k)}

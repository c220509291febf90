"""Barycentric distance and Expected Barycenter Effect (oracle, float64).

Paper, Sec. "Geodesic Sinkhorn Distances": gamma(T, C) = W(mu*_T, mu*_C), the
Geodesic Sinkhorn distance between the barycenters of the two families, and
tau(T) = E_{mu*_T}(Y) - E_{mu*_C}(Y), the difference of the feature
expectations under the two barycenters (computed in closed form as weighted
means over the nodes).  Reading: the barycenters enter Algorithm 1 as
computed (unit mass up to convergence); an expectation divides by the mass.
"""
from __future__ import annotations

import numpy as np

from .sinkhorn import barycenter, sinkhorn


def expectation(p, Y) -> np.ndarray:
    """sum_i p_i Y_i / sum_i p_i (Y of shape (n,) or (n, d))."""
    p = np.asarray(p, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64).reshape(p.shape[0], -1)
    return (p @ Y) / p.sum()


def barycentric_distance(L, lam_hat, t, K, fam_T, alpha_T, fam_C, alpha_C, iters_bary, iters_sinkhorn):
    """(gamma, p_T, p_C)."""
    p_T = barycenter(L, lam_hat, t, K, fam_T, alpha_T, iters_bary)["p"]
    p_C = barycenter(L, lam_hat, t, K, fam_C, alpha_C, iters_bary)["p"]
    D = sinkhorn(L, lam_hat, t, K, p_T, p_C, iters_sinkhorn, marginals=False)["D"][0]
    return float(D), p_T, p_C


def expected_barycenter_effect(p_T, p_C, Y) -> np.ndarray:
    return expectation(p_T, Y) - expectation(p_C, Y)

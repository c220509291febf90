"""Distances and effects between families of distributions (library calls only).

Paper, Sec. "Geodesic Sinkhorn Distances": the barycentric distance between
two finite families T and C on the common graph is the Geodesic Sinkhorn
distance between their barycenters, gamma(T, C) = W(mu*_T, mu*_C); the
Expected Barycenter Effect is tau(T) = E_{mu*_T}(Y) - E_{mu*_C}(Y), the
difference of the feature expectations under the two barycenters.  Every
numerical step runs in libgeosink: gs_barycenter for each family,
gs_sinkhorn for the distance between the barycenters, gs_expectation for the
feature means.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Graph, Plan, gs_barycenter, gs_expectation, gs_sinkhorn


def family_barycenter(graph: Graph, lambda_hat: float, t: float, K: int, mus: torch.Tensor, alpha, iters: int,
                      phi: float = 1e-30) -> torch.Tensor:
    """Barycenter (n,) of the family given as the columns of mus (n, m)."""
    m = mus.shape[1]
    plan = Plan(graph, K, m)
    bary = torch.empty(graph.n, device=mus.device, dtype=torch.float32)
    gs_barycenter(plan, lambda_hat, t, mus.contiguous(), np.asarray(alpha, dtype=np.float64), iters, bary, phi=phi)
    return bary


def barycentric_distance(graph: Graph, lambda_hat: float, t: float, K: int, fam_T: torch.Tensor, alpha_T,
                         fam_C: torch.Tensor, alpha_C, iters_bary: int, iters_sinkhorn: int, phi: float = 1e-30):
    """gamma(T, C): returns (distance D between the barycenters, p_T, p_C).

    D is Algorithm 1's return value with the two barycenters as the two
    distributions (taken as computed: iterative Bregman projections give them
    unit mass up to their convergence).
    """
    p_T = family_barycenter(graph, lambda_hat, t, K, fam_T, alpha_T, iters_bary, phi)
    p_C = family_barycenter(graph, lambda_hat, t, K, fam_C, alpha_C, iters_bary, phi)
    plan = Plan(graph, K, 1)
    out = gs_sinkhorn(plan, lambda_hat, t, p_T, p_C, iters_sinkhorn, phi=phi)
    return float(out["dist"][0]), p_T, p_C


def expected_barycenter_effect(p_T: torch.Tensor, p_C: torch.Tensor, Y: torch.Tensor) -> np.ndarray:
    """tau = E_{p_T}(Y) - E_{p_C}(Y) for node features Y (n,) or (n, d)."""
    return gs_expectation(p_T, Y) - gs_expectation(p_C, Y)

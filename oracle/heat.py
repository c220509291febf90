"""Chebyshev approximation of the graph heat kernel (oracle, float64).

Paper, Sec. "Heat Diffusion on a Graph": H_t = exp(-t L) = Psi exp(-t Lambda)
Psi^T; only its application to a signal is needed.  Sec. "Chebyshev
Polynomials": H_t = b_0/2 + sum_{k>=1} b_k T_k(L - Id) under lambda_n <= 2,
with Bessel-function coefficients, truncated at degree K to p_K(L, t), which
costs K sparse matrix-vector products.

Readings used here:
  * the operator is rescaled, L_op = (2/lam_hat) L with lam_hat >= lambda_max,
    and t is the time on L_op: H_t := exp(-t L_op), y := L_op - I, so the
    paper's T_k(L - Id) is literally T_k(y);
  * T_0 = 1 (the printed T_0 = 0 is a typo: the recurrence needs T_0 = 1);
  * degree K means coefficients b_0..b_K and K products, with b_0 halved;
  * the Bessel coefficients come from the generating function
    exp(z cos th) = I_0(z) + 2 sum_k I_k(z) cos(k th) at z = -t, giving
    exp(-t(y+1)) = sum' b_k T_k(y) with b_k = 2 (-1)^k exp(-t) I_k(t).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu
from scipy.special import ive


def cheb_coeffs(t: float, K: int) -> np.ndarray:
    """b_k = 2 (-1)^k e^{-t} I_k(t), k = 0..K (b_0 is NOT halved here)."""
    k = np.arange(K + 1)
    return 2.0 * (-1.0) ** k * ive(k, t)


def cheb_coeffs_dt(t: float, K: int) -> np.ndarray:
    """d b_k / dt = 2 (-1)^k e^{-t} (I_k'(t) - I_k(t)), with I_k' = (I_{k-1} + I_{k+1}) / 2.

    I_{-1} = I_1 for integer order.
    """
    k = np.arange(K + 1)
    ik = ive(k, t)
    ikm1 = ive(np.abs(k - 1), t)
    ikp1 = ive(k + 1, t)
    return 2.0 * (-1.0) ** k * (0.5 * (ikm1 + ikp1) - ik)


def tail_bound(t: float, K: int, extra: int = 400) -> float:
    """sum_{k>K} |b_k|: bound on sup_{y in [-1,1]} |p_K(y) - exp(-t(y+1))|."""
    k = np.arange(K + 1, K + 1 + extra)
    return float(np.sum(2.0 * ive(k, t)))


def rescaled_operator(L: sp.spmatrix, lam_hat: float) -> sp.csr_matrix:
    """y = (2/lam_hat) L - I, spectrum in [-1, 1] when lam_hat >= lambda_max."""
    n = L.shape[0]
    return (sp.csr_matrix(L, dtype=np.float64) * (2.0 / lam_hat) - sp.identity(n, format="csr")).tocsr()


def _cheb_sum(L, lam_hat, coef, X):
    """sum' coef_k T_k(y) X via the three-term recurrence (K products with y)."""
    y = rescaled_operator(L, lam_hat)
    X = np.asarray(X, dtype=np.float64)
    K = len(coef) - 1
    t_prev = X                      # T_0 x
    out = 0.5 * coef[0] * t_prev
    if K == 0:
        return out
    t_cur = y @ X                   # T_1 x
    out = out + coef[1] * t_cur
    for k in range(2, K + 1):
        t_next = 2.0 * (y @ t_cur) - t_prev
        out = out + coef[k] * t_next
        t_prev, t_cur = t_cur, t_next
    return out


def heat_apply(L, lam_hat: float, t: float, K: int, X) -> np.ndarray:
    """p_K(L, t) X for X of shape (n,) or (n, B)."""
    return _cheb_sum(L, lam_hat, cheb_coeffs(t, K), X)


def heat_apply_dt(L, lam_hat: float, t: float, K: int, X) -> np.ndarray:
    """(d/dt) p_K(L, t) X = sum' b_k'(t) T_k(y) X."""
    return _cheb_sum(L, lam_hat, cheb_coeffs_dt(t, K), X)


def heat_dense_exact(L, lam_hat: float, t: float) -> np.ndarray:
    """exp(-t (2/lam_hat) L) by dense eigendecomposition (tiny n only)."""
    Ld = L.toarray() if sp.issparse(L) else np.asarray(L, dtype=np.float64)
    lam, psi = np.linalg.eigh(Ld)
    return (psi * np.exp(-t * (2.0 / lam_hat) * lam)) @ psi.T


def heat_dense_poly(L, lam_hat: float, t: float, K: int) -> np.ndarray:
    """The dense matrix p_K(L, t) (tiny n only)."""
    n = L.shape[0]
    return heat_apply(L, lam_hat, t, K, np.eye(n))


def euler_apply(L, lam_hat: float, t: float, N: int, X) -> np.ndarray:
    """(I + (t/N) L_op)^{-N} X: N backward-Euler steps of the heat equation.

    Paper, Sec. "Related work" (heat kernel applied by solving linear systems
    of the discretised heat equation) and the ground cost of the Euler
    discretisation next to Proposition "ground cost": with the sign typo read
    as (I + (t/N) L_op)^{-N}, eps = 4t, and L_op = (2/lam_hat) L as for the
    Chebyshev kernel.  Each step is an exact sparse LU solve.
    """
    n = L.shape[0]
    A = (sp.identity(n, format="csc") + (t / N) * (2.0 / lam_hat) * sp.csc_matrix(L, dtype=np.float64)).tocsc()
    lu = splu(A)
    Y = np.asarray(X, dtype=np.float64)
    for _ in range(N):
        Y = lu.solve(Y)
    return Y

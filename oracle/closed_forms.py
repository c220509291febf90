"""Closed forms of the heat-kernel polynomial and of tiny transport problems.

These evaluate the same quantities as heat.py / sinkhorn.py by independent
routes (spectral diagonalisation by FFT, T_k(y) = cos(k arccos y), exact
two-node formulas, one-dimensional convex minimisation), so that the recurrence
code is checked against something other than itself, and so that GPU results
at sizes the sparse oracle cannot reach are still compared with an exact value.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize_scalar

from .heat import cheb_coeffs


def poly_at_eigs(lams: np.ndarray, lam_hat: float, t: float, K: int) -> np.ndarray:
    """Scalar p_K at Laplacian eigenvalues lams: sum' b_k cos(k arccos y), y = 2 lam / lam_hat - 1."""
    y = np.clip(2.0 * np.asarray(lams, dtype=np.float64) / lam_hat - 1.0, -1.0, 1.0)
    th = np.arccos(y)
    b = cheb_coeffs(t, K)
    k = np.arange(K + 1)
    terms = b[None, :] * np.cos(np.outer(th.ravel(), k))
    terms[:, 0] *= 0.5
    return terms.sum(axis=1).reshape(np.shape(lams))


def euler_at_eigs(lams: np.ndarray, lam_hat: float, t: float, N: int) -> np.ndarray:
    """Backward-Euler kernel at Laplacian eigenvalues: (1 + (t/N)(2/lam_hat) lam)^{-N}."""
    return (1.0 + (t / N) * (2.0 / lam_hat) * np.asarray(lams, dtype=np.float64)) ** (-N)


def cycle_euler_apply(n: int, lam_hat: float, t: float, N: int, X: np.ndarray) -> np.ndarray:
    """(I + (t/N) L_op)^{-N} X on the cycle through its Fourier diagonalisation."""
    X = np.asarray(X, dtype=np.float64)
    p = euler_at_eigs(cycle_eigs(n), lam_hat, t, N)
    shape = (n,) + (1,) * (X.ndim - 1)
    return np.real(np.fft.ifft(p.reshape(shape) * np.fft.fft(X, axis=0), axis=0))


def cycle_eigs(n: int) -> np.ndarray:
    """Eigenvalues 2 - 2 cos(2 pi j / n) of the unit-weight cycle Laplacian (FFT order)."""
    return 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)


def cycle_heat_apply(n: int, lam_hat: float, t: float, K: int, X: np.ndarray) -> np.ndarray:
    """p_K(L(C_n), t) X through the Fourier diagonalisation of the cycle."""
    X = np.asarray(X, dtype=np.float64)
    p = poly_at_eigs(cycle_eigs(n), lam_hat, t, K)
    Xh = np.fft.fft(X, axis=0)
    shape = (n,) + (1,) * (X.ndim - 1)
    return np.real(np.fft.ifft(p.reshape(shape) * Xh, axis=0))


def torus_heat_apply(n1: int, n2: int, lam_hat: float, t: float, K: int, X: np.ndarray) -> np.ndarray:
    """p_K(L(C_n1 x C_n2), t) X, node id a*n2 + b; X is (n1*n2,) or (n1*n2, B)."""
    X = np.asarray(X, dtype=np.float64)
    tail = X.shape[1:]
    Xg = X.reshape((n1, n2) + tail)
    lam = cycle_eigs(n1)[:, None] + cycle_eigs(n2)[None, :]
    p = poly_at_eigs(lam, lam_hat, t, K).reshape((n1, n2) + (1,) * len(tail))
    Y = np.real(np.fft.ifft2(p * np.fft.fft2(Xg, axes=(0, 1)), axes=(0, 1)))
    return Y.reshape(X.shape)


def complete_heat_apply(n: int, t: float, K: int, X: np.ndarray) -> np.ndarray:
    """p_K for the unit complete graph K_n with lam_hat = n (spectrum {0, n})."""
    X = np.asarray(X, dtype=np.float64)
    p0, pn = poly_at_eigs(np.array([0.0, float(n)]), float(n), t, K)
    mean = X.mean(axis=0, keepdims=True)
    return p0 * mean + pn * (X - mean)


def two_node_kernel(t: float, K: int | None = None, weight: float = 1.0) -> np.ndarray:
    """2x2 heat kernel of one edge of weight `weight` with lam_hat = 2*weight.

    Eigenvalues 0 (vector (1,1)) and 2*weight (vector (1,-1)); after
    rescaling they sit at y = -1 and y = +1.  K=None gives the exact kernel.
    """
    if K is None:
        s, c = 1.0, np.exp(-2.0 * t)
    else:
        s, c = poly_at_eigs(np.array([0.0, 2.0 * weight]), 2.0 * weight, t, K)
    return 0.5 * np.array([[s + c, s - c], [s - c, s + c]])


def two_node_dirac_distance(t: float, K: int | None = None) -> float:
    """D(delta_1, delta_2) on one edge: the only coupling moves all mass 1 -> 2, so D = -4t ln H_12."""
    H = two_node_kernel(t, K)
    return float(-4.0 * t * np.log(H[0, 1]))


def two_node_plan_cost(H: np.ndarray, mu: np.ndarray, nu: np.ndarray) -> float:
    """min over 2x2 couplings pi of mu, nu of sum pi ln(pi / H), by 1-D convex minimisation.

    pi = [[s, mu0 - s], [nu0 - s, 1 - mu0 - nu0 + s]] (unit total mass).
    Returns the minimum (Algorithm 1's D divided by 4t).
    """
    mu0, nu0 = float(mu[0]), float(nu[0])
    lo = max(0.0, mu0 + nu0 - 1.0)
    hi = min(mu0, nu0)

    def f(s):
        pi = np.array([s, mu0 - s, nu0 - s, 1.0 - mu0 - nu0 + s])
        h = np.array([H[0, 0], H[0, 1], H[1, 0], H[1, 1]])
        pos = pi > 0
        return float(np.sum(pi[pos] * np.log(pi[pos] / h[pos])))

    if hi - lo < 1e-15:
        return f(lo)
    res = minimize_scalar(f, bounds=(lo, hi), method="bounded",
                          options={"xatol": 1e-14, "maxiter": 2000})
    return float(res.fun)


def two_node_barycenter(H: np.ndarray, mus: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """Fixed-support barycenter on two nodes: argmin_p sum_i alpha_i min_pi KL(pi | H), by nested 1-D search."""
    def F(p0):
        p = np.array([p0, 1.0 - p0])
        return sum(al * two_node_plan_cost(H, mus[:, i], p) for i, al in enumerate(alpha))

    res = minimize_scalar(F, bounds=(1e-9, 1.0 - 1e-9), method="bounded",
                          options={"xatol": 1e-12, "maxiter": 2000})
    return np.array([res.x, 1.0 - res.x])


def dual_ascent_distance(Hmat: np.ndarray, mu: np.ndarray, nu: np.ndarray) -> float:
    """Entropic OT value sum pi ln(pi / H) at the optimum, from the dual by L-BFGS.

    maximise <mu, f> + <nu, g> - sum_ij H_ij e^{f_i + g_j} + 1 over (f, g) on the
    supports; at the optimum pi = diag(e^f) H diag(e^g) has the right marginals
    and the dual value equals the primal sum pi ln(pi / H) for unit masses.
    A route independent of Sinkhorn's fixed-point updates.
    """
    from scipy.optimize import minimize

    si = np.nonzero(mu > 0)[0]
    sj = np.nonzero(nu > 0)[0]
    Hs = Hmat[np.ix_(si, sj)]
    m0, n0 = mu[si], nu[sj]

    def neg(z):
        f, g = z[:len(si)], z[len(si):]
        P = Hs * np.exp(f[:, None] + g[None, :])
        val = m0 @ f + n0 @ g - P.sum() + 1.0
        grad = np.concatenate([m0 - P.sum(axis=1), n0 - P.sum(axis=0)])
        return -val, -grad

    z0 = np.concatenate([np.log(m0), np.log(n0)])
    res = minimize(neg, z0, jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "gtol": 1e-13, "ftol": 1e-16})
    return float(-res.fun)

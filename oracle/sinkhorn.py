"""Geodesic Sinkhorn distance, barycenter and gradient (oracle, float64).

Paper: Algorithm 1 (Geodesic Sinkhorn) with the heat-kernel approximation
p_K(L, t) of Sec. "Chebyshev Polynomials"; the entropic OT background of Sec.
"Sinkhorn Distances" (plan diag(v) K diag(w), updates v <- mu / K w,
w <- nu / K^T v); Varadhan's formula giving lambda = 4t; the fixed-support
barycenter of Sec. "Interpolation with discrete support".

Readings used here:
  * Algorithm 1 takes t directly (its "regularization lambda" is 4t);
  * vertex weights a default to all ones;
  * w starts at ones, v is updated before w, a fixed number J of iterations
    is run (no stopping rule is given);
  * the returned value is the expression on Algorithm 1's return line,
    D = 4t sum a (mu ln v + nu ln w) = 4t (1 + min KL) at the fixed point
    (the entropic cost itself, not its square root);
  * 0 ln 0 = 0 (the sums run over the supports);
  * denominators are floored, d = r if r > phi else phi, phi = 1e-30, and
    floored entries on the numerator's support are counted;
  * the barycenter algorithm is not given in the paper: iterative Bregman
    projections (Benamou et al. 2015) in the form
    v_i = mu_i / p_K(a w_i), q_i = p_K(a v_i), p = exp(sum_i alpha_i ln q_i),
    w_i = p / q_i, starting from w_i = 1;
  * gradients are taken through exactly J unrolled iterations with
    d floor(r)/dr = 1[r > phi]; lam_hat is held fixed.
Signals may be (n,) or (n, B); every column is an independent problem.
"""
from __future__ import annotations

import numpy as np

from .heat import heat_apply, heat_apply_dt

PHI = 1e-30


def _floor(r, phi):
    mask = r > phi
    return np.where(mask, r, phi), mask


def _xlogy_support(x, y):
    """x * ln y where x > 0, else 0."""
    out = np.zeros(np.broadcast(x, y).shape)
    s = x > 0
    out[s] = x[s] * np.log(y[s])
    return out


def _as2d(x):
    x = np.asarray(x, dtype=np.float64)
    return (x[:, None], True) if x.ndim == 1 else (x, False)


def sinkhorn(L, lam_hat, t, K, mu, nu, J, a=None, phi=PHI, record=False, marginals=True, apply=None):
    """Algorithm 1.  Returns a dict with D (B,), v, w, marginal errors and floor counts.

    marg_row = ||a v p_K(a w) - a mu||_1 (one extra heat application),
    marg_col = ||a w p_K(a v) - a nu||_1 (zero up to floors).
    `apply` (x -> H x) replaces p_K by another symmetric kernel (e.g. the
    backward-Euler one); L, lam_hat and K are then unused.
    """
    mu, squeeze = _as2d(mu)
    nu, _ = _as2d(nu)
    n, B = mu.shape
    a = np.ones(n) if a is None else np.asarray(a, dtype=np.float64)
    ac = a[:, None]
    H = apply if apply is not None else (lambda x: heat_apply(L, lam_hat, t, K, x))
    w = np.ones((n, B))
    v = np.zeros((n, B))
    n_floored = 0
    rec = {"d": [], "e": [], "rmask": [], "emask": []} if record else None
    for _ in range(J):
        d, dm = _floor(H(ac * w), phi)
        v = mu / d
        e, em = _floor(H(ac * v), phi)
        w = nu / e
        n_floored += int(np.sum((~dm) & (mu > 0)) + np.sum((~em) & (nu > 0)))
        if record:
            rec["d"].append(d)
            rec["e"].append(e)
            rec["rmask"].append(dm)
            rec["emask"].append(em)
    D = 4.0 * t * np.sum(ac * (_xlogy_support(mu, v) + _xlogy_support(nu, w)), axis=0)
    out = {"D": D, "v": v, "w": w, "n_floored": n_floored}
    if marginals:
        out["marg_row"] = np.sum(np.abs(ac * v * H(ac * w) - ac * mu), axis=0)
        out["marg_col"] = np.sum(np.abs(ac * w * H(ac * v) - ac * nu), axis=0)
    if record:
        out["record"] = rec
    if squeeze:
        for key in ("v", "w"):
            out[key] = out[key][:, 0]
    return out


def row_marginal(L, lam_hat, t, K, v, w, a=None):
    """a v p_K(a w): the plan's row marginal, evaluated in float64."""
    v, _ = _as2d(v)
    w, _ = _as2d(w)
    a = np.ones(v.shape[0]) if a is None else np.asarray(a, dtype=np.float64)
    ac = a[:, None]
    return ac * v * heat_apply(L, lam_hat, t, K, ac * w)


def barycenter(L, lam_hat, t, K, mus, alpha, J, a=None, phi=PHI, apply=None):
    """Fixed-support barycenter by iterative Bregman projections.

    mus (n, m), alpha (m,).  Returns dict with p (n,), v, w (n, m) and the
    per-input row-marginal errors ||a v_i p_K(a w_i) - a mu_i||_1.  `apply`
    replaces p_K as in `sinkhorn`.
    """
    mus = np.asarray(mus, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    n, m = mus.shape
    a = np.ones(n) if a is None else np.asarray(a, dtype=np.float64)
    ac = a[:, None]
    H = apply if apply is not None else (lambda x: heat_apply(L, lam_hat, t, K, x))
    w = np.ones((n, m))
    v = np.zeros((n, m))
    p = np.zeros(n)
    n_floored = 0
    for _ in range(J):
        d, dm = _floor(H(ac * w), phi)
        v = mus / d
        q, qm = _floor(H(ac * v), phi)
        p = np.exp(np.log(q) @ alpha)
        w = p[:, None] / q
        n_floored += int(np.sum((~dm) & (mus > 0)) + np.sum(~qm))
    marg = np.sum(np.abs(ac * v * H(ac * w) - ac * mus), axis=0)
    return {"p": p, "v": v, "w": w, "marg_row": marg, "n_floored": n_floored}


def sinkhorn_grad(L, lam_hat, t, K, mu, nu, J, a=None, phi=PHI, g=None):
    """Reverse-mode gradient of D (Algorithm 1's output) through J iterations.

    g (B,) weights the columns (default ones).  Returns dict with D, dmu, dnu
    (n, B; reported on the supports, zero elsewhere) and dt (B,).
    Uses p_K^T = p_K and (d/dt p_K)^T = d/dt p_K (polynomials in symmetric L).
    """
    mu, squeeze = _as2d(mu)
    nu, _ = _as2d(nu)
    n, B = mu.shape
    a = np.ones(n) if a is None else np.asarray(a, dtype=np.float64)
    ac = a[:, None]
    g = np.ones(B) if g is None else np.asarray(g, dtype=np.float64)
    H = lambda x: heat_apply(L, lam_hat, t, K, x)
    Hd = lambda x: heat_apply_dt(L, lam_hat, t, K, x)

    # forward, keeping every iterate
    ws = [np.ones((n, B))]
    vs, ds, es, dms, ems = [None], [None], [None], [None], [None]
    for _ in range(J):
        d, dm = _floor(H(ac * ws[-1]), phi)
        v = mu / d
        e, em = _floor(H(ac * v), phi)
        w = nu / e
        vs.append(v); ds.append(d); dms.append(dm)
        es.append(e); ems.append(em); ws.append(w)
    vJ, wJ = vs[J], ws[J]
    S = np.sum(ac * (_xlogy_support(mu, vJ) + _xlogy_support(nu, wJ)), axis=0)
    D = 4.0 * t * S

    # seeds from D = 4t sum a (mu ln v + nu ln w)
    smu, snu = mu > 0, nu > 0
    dmu = np.where(smu, 4.0 * t * ac * np.log(np.where(smu, vJ, 1.0)), 0.0)
    dnu = np.where(snu, 4.0 * t * ac * np.log(np.where(snu, wJ, 1.0)), 0.0)
    vbar = np.where(smu, 4.0 * t * ac * mu / np.where(smu, vJ, 1.0), 0.0)
    wbar = np.where(snu, 4.0 * t * ac * nu / np.where(snu, wJ, 1.0), 0.0)
    dt = S * 4.0  # explicit d/dt of the 4t prefactor, = D / t

    for j in range(J, 0, -1):
        # w_j = nu / e_j,  e_j = floor(p_K(a v_j))
        dnu = dnu + wbar / es[j]
        ebar = -wbar * ws[j] / es[j] * ems[j]
        vbar = vbar + ac * H(ebar)
        dt = dt + np.sum(Hd(ebar) * ac * vs[j], axis=0)
        # v_j = mu / d_j,  d_j = floor(p_K(a w_{j-1}))
        dmu = dmu + vbar / ds[j]
        dbar = -vbar * vs[j] / ds[j] * dms[j]
        wbar = ac * H(dbar)
        dt = dt + np.sum(Hd(dbar) * ac * ws[j - 1], axis=0)
        vbar = np.zeros_like(vbar)

    dmu = np.where(smu, dmu, 0.0) * g
    dnu = np.where(snu, dnu, 0.0) * g
    out = {"D": D, "dmu": dmu, "dnu": dnu, "dt": dt * g}
    if squeeze:
        out["dmu"], out["dnu"] = dmu[:, 0], dnu[:, 0]
    return out


def finite_diff_mu(L, lam_hat, t, K, mu, nu, J, coords, rel_step=1e-4, a=None, phi=PHI):
    """Central differences of D w.r.t. mu[i] with step rel_step * mu[i] (single pair)."""
    mu = np.asarray(mu, dtype=np.float64)
    out = []
    for i in coords:
        h = rel_step * mu[i]
        mp, mm = mu.copy(), mu.copy()
        mp[i] += h
        mm[i] -= h
        Dp = sinkhorn(L, lam_hat, t, K, mp, nu, J, a=a, phi=phi, marginals=False)["D"][0]
        Dm = sinkhorn(L, lam_hat, t, K, mm, nu, J, a=a, phi=phi, marginals=False)["D"][0]
        out.append((Dp - Dm) / (2.0 * h))
    return np.array(out)


def finite_diff_t(L, lam_hat, t, K, mu, nu, J, h=1e-4, a=None, phi=PHI):
    """Central difference of D w.r.t. t with absolute step h."""
    Dp = sinkhorn(L, lam_hat, t + h, K, mu, nu, J, a=a, phi=phi, marginals=False)["D"]
    Dm = sinkhorn(L, lam_hat, t - h, K, mu, nu, J, a=a, phi=phi, marginals=False)["D"]
    return (Dp - Dm) / (2.0 * h)

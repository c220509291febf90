"""Float64 oracle values for the GPU parity tests at each workload's own size and length.

    python tests/golden/make_fullsize.py [curve] [bary] [grad] [local1m] [--procs 6]

Calls only `oracle/` (the float64 reference) and `synth/` (seeded inputs);
nothing here loads the GPU library.  For every workload it writes
`tests/golden/fullsize_<name>.json` (input digests, lambda values, distances,
marginal errors, t-gradients, finite differences) and
`tests/golden/fullsize_<name>.npz` (float32 arrays restricted to the
histograms' supports, in ascending node order: row marginals, barycenters,
gradients).  The GPU tests rebuild the same inputs, check the digests, and
compare against these values.

Workloads (paper: Algorithm 1 run for J iterations with the Chebyshev heat
kernel of Sec. "Chebyshev Polynomials"; the barycenter of Sec.
"Interpolation with discrete support"; the gradients through the unrolled
iterations):
  curve    n = 100k (20 clusters on a curve in R^50, k = 15), one pair,
           K = 30, J = 500, t in {0.5, 2, 8}
  bary     n = 200k (30 clusters, k = 15), m = 64, K = 40, t = 2: the first
           20 iterations at full size, and all 300 iterations on the
           n = 20k twin of the same recipe (supports scaled by 1/10)
  grad     the n = 200k graph, 32 pairs, K = 30, t = 2, J = 200: reference
           gradients of pairs 0-3 and central differences (relative steps
           1e-4 and 1e-3) on 16 support coordinates (4 per pair) and in t
  local1m  n = 1M random local graph with the 1M kNN workload's size
           (18.4M nonzeros, 200 hubs), 32 pairs of log-uniform supports
           [5k, 200k], K = 50, t = 2, J = 200: the two pairs with the
           smallest supports, forward and reverse sweep

The kNN graphs are the oracle's own (brute force, split over processes by
row ranges); lambda_hat = 1.01 lambda_max(L) from ARPACK on the float32
weights the GPU also uses, and the same lambda_hat is given to both sides.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import graph as ograph  # noqa: E402
from oracle import sinkhorn as osk  # noqa: E402
from oracle import spectrum  # noqa: E402

STATE = {}   # graphs and inputs, inherited by the forked workers


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _knn_rows(args):
    lo, hi, k = args
    return ograph.knn_lists(STATE["X"], k, rows=(lo, hi))[0]


def oracle_graph(X, k, procs):
    """The oracle's kNN graph of X with float32 weights, plus its description."""
    n = X.shape[0]
    STATE["X"] = X
    step = max(512, -(-n // (procs * 8)) // 512 * 512)
    ranges = [(lo, min(n, lo + step), k) for lo in range(0, n, step)]
    with mp.get_context("fork").Pool(procs) as pool:
        idx = np.concatenate(pool.map(_knn_rows, ranges), axis=0)
    A64, info = ograph.knn_graph(X, k, knn_idx=idx)
    rp = A64.indptr.astype(np.int32)
    col = A64.indices.astype(np.int32)
    w32 = A64.data.astype(np.float32)
    return graph_record(n, rp, col, w32, extra={"k": k, "median": info["median"], "n_components": info["n_components"]})


def graph_record(n, rp, col, w32, extra=None):
    A = ograph.csr_from_arrays(n, rp, col, w32.astype(np.float64))
    L = ograph.laplacian(A)
    t0 = time.perf_counter()
    lmax = spectrum.lambda_max(L)
    rec = {"n": int(n), "nnz": int(col.shape[0]), "rowptr_sha256": synth.sha256(rp), "col_sha256": synth.sha256(col),
           "w_sha256": synth.sha256(w32), "lambda_max": lmax, "lambda_hat": 1.01 * lmax,
           "edge_bound": spectrum.edge_bound(A), "lambda_max_seconds": round(time.perf_counter() - t0, 1)}
    rec.update(extra or {})
    return L, rec


def on_support(x, s):
    return np.asarray(x, dtype=np.float64)[s].astype(np.float32)


# ----------------------------------------------------------------------------- jobs (run in forked workers)

def job_curve(t):
    L, g = STATE["curve_L"], STATE["curve_graph"]
    mu, nu = STATE["curve_mu"], STATE["curve_nu"]
    K, J = 30, 500
    t0 = time.perf_counter()
    r = osk.sinkhorn(L, g["lambda_hat"], t, K, mu, nu, J)
    row = osk.row_marginal(L, g["lambda_hat"], t, K, r["v"], r["w"])[:, 0]
    log(f"curve t={t} D={r['D'][0]:.10g} marg_row={r['marg_row'][0]:.3e} ({time.perf_counter() - t0:.0f}s)")
    return {"t": t, "D": float(r["D"][0]), "marg_row": float(r["marg_row"][0]), "marg_col": float(r["marg_col"][0]),
            "n_floored": int(r["n_floored"]), "row_marginal": on_support(row, mu > 0)}


def job_bary(which):
    L, g, H = STATE[f"{which}_L"], STATE[f"{which}_graph"], STATE[f"{which}_H"]
    K, t, J = 40, 2.0, STATE[f"{which}_J"]
    m = H.shape[1]
    t0 = time.perf_counter()
    r = osk.barycenter(L, g["lambda_hat"], t, K, H.astype(np.float64), np.full(m, 1.0 / m), J)
    log(f"{which} J={J} mass={r['p'].sum():.9f} ({time.perf_counter() - t0:.0f}s)")
    return {"J": J, "p": r["p"].astype(np.float32), "mass": float(r["p"].sum()),
            "marg_row": [float(x) for x in r["marg_row"]], "n_floored": int(r["n_floored"])}


def job_grad_ref(c):
    L, g = STATE["bary_L"], STATE["bary_graph"]
    mu, nu = STATE["grad_mu"][:, [c]].astype(np.float64), STATE["grad_nu"][:, [c]].astype(np.float64)
    K, t, J = 30, 2.0, 200
    t0 = time.perf_counter()
    r = osk.sinkhorn_grad(L, g["lambda_hat"], t, K, mu, nu, J)
    f = osk.sinkhorn(L, g["lambda_hat"], t, K, mu, nu, J)
    row = osk.row_marginal(L, g["lambda_hat"], t, K, f["v"], f["w"])
    log(f"grad ref pair {c} D={r['D'][0]:.10g} ({time.perf_counter() - t0:.0f}s)")
    at_fd = [float(r["dmu"][i, 0]) for cc, i in STATE["grad_spec"] if cc == c]
    return {"D": float(f["D"][0]), "D_grad_run": float(r["D"][0]), "dt": float(r["dt"][0]),
            "marg_row": float(f["marg_row"][0]), "n_floored": int(f["n_floored"]), "dmu_at_fd": at_fd,
            "dmu": on_support(r["dmu"][:, 0], mu[:, 0] > 0), "dnu": on_support(r["dnu"][:, 0], nu[:, 0] > 0),
            "row": on_support(row[:, 0], mu[:, 0] > 0)}


def job_grad_fd(args):
    """Central differences of D in mu at (pair, node) coordinates, one column per perturbation.

    Relative step 1e-4 (the workload's step) and 1e-3: float64 rounding of D
    (about 20 ulp after J = 200 iterations) divided by the step dominates the
    first where mu_i is small (up to 1e-5 relative); the larger step cuts that
    tenfold at a truncation error of about 1e-8 relative.
    """
    spec, rel = args
    L, g = STATE["bary_L"], STATE["bary_graph"]
    K, t, J = 30, 2.0, 200
    mu0, nu0 = STATE["grad_mu"].astype(np.float64), STATE["grad_nu"].astype(np.float64)
    n = mu0.shape[0]
    cols_mu, cols_nu, steps = [], [], []
    for c, i in spec:
        h = rel * mu0[i, c]
        mp_, mm_ = mu0[:, c].copy(), mu0[:, c].copy()
        mp_[i] += h
        mm_[i] -= h
        cols_mu += [mp_, mm_]
        cols_nu += [nu0[:, c], nu0[:, c]]
        steps.append(mp_[i] - mm_[i])    # the step as represented (2h up to rounding)
    t0 = time.perf_counter()
    D = osk.sinkhorn(L, g["lambda_hat"], t, K, np.stack(cols_mu, axis=1), np.stack(cols_nu, axis=1), J,
                     marginals=False)["D"]
    log(f"grad fd {len(spec)} coordinates, relative step {rel} ({time.perf_counter() - t0:.0f}s)")
    assert n == mu0.shape[0]
    return [{"pair": int(c), "node": int(i), "rel": rel, "h": float(h / 2), "fd": float((D[2 * q] - D[2 * q + 1]) / h)}
            for q, ((c, i), h) in enumerate(zip(spec, steps))]


def job_grad_fd_t(c):
    L, g = STATE["bary_L"], STATE["bary_graph"]
    K, t, J, h = 30, 2.0, 200, 1e-4
    mu, nu = STATE["grad_mu"][:, [c]].astype(np.float64), STATE["grad_nu"][:, [c]].astype(np.float64)
    t0 = time.perf_counter()
    Dp = osk.sinkhorn(L, g["lambda_hat"], t + h, K, mu, nu, J, marginals=False)["D"][0]
    Dm = osk.sinkhorn(L, g["lambda_hat"], t - h, K, mu, nu, J, marginals=False)["D"][0]
    log(f"grad fd t pair {c} ({time.perf_counter() - t0:.0f}s)")
    return float((Dp - Dm) / (2.0 * h))


def job_local1m(c):
    L, g = STATE["local1m_L"], STATE["local1m_graph"]
    mu, nu = STATE["local1m_mu"][:, [c]].astype(np.float64), STATE["local1m_nu"][:, [c]].astype(np.float64)
    K, t, J = 50, 2.0, 200
    t0 = time.perf_counter()
    r = osk.sinkhorn_grad(L, g["lambda_hat"], t, K, mu, nu, J)
    log(f"local1m pair {c} gradient D={r['D'][0]:.10g} ({time.perf_counter() - t0:.0f}s)")
    f = osk.sinkhorn(L, g["lambda_hat"], t, K, mu, nu, J)
    row = osk.row_marginal(L, g["lambda_hat"], t, K, f["v"], f["w"])
    log(f"local1m pair {c} forward marg_row={f['marg_row'][0]:.3e} ({time.perf_counter() - t0:.0f}s)")
    return {"D": float(f["D"][0]), "D_grad_run": float(r["D"][0]), "dt": float(r["dt"][0]),
            "marg_row": float(f["marg_row"][0]), "marg_col": float(f["marg_col"][0]), "n_floored": int(f["n_floored"]),
            "dmu": on_support(r["dmu"][:, 0], mu[:, 0] > 0), "dnu": on_support(r["dnu"][:, 0], nu[:, 0] > 0),
            "row": on_support(row[:, 0], mu[:, 0] > 0)}


def run_job(job):
    name, arg = job
    return name, arg, globals()[name](arg)


# ----------------------------------------------------------------------------- main

def split_arrays(res):
    """(json part, arrays part) of a job result."""
    if isinstance(res, dict):
        js = {k: v for k, v in res.items() if not isinstance(v, np.ndarray)}
        arr = {k: v for k, v in res.items() if isinstance(v, np.ndarray)}
        return js, arr
    return res, {}


def save(name, record, arrays):
    with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as f:
        json.dump(record, f, indent=1, sort_keys=True)
    np.savez_compressed(os.path.join(HERE, f"fullsize_{name}.npz"), **arrays)
    log(f"wrote fullsize_{name}.json / .npz ({len(arrays)} arrays)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+", choices=["curve", "bary", "grad", "local1m"])
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    jobs = []
    records = {}
    if "curve" in args.which:
        X, labels, mu, nu = synth.curve_pair_workload()
        log(f"curve: building the oracle graph of {X.shape}")
        L, g = oracle_graph(X, 15, args.procs)
        log(f"curve graph {g}")
        STATE.update(curve_L=L, curve_graph=g, curve_mu=mu.astype(np.float64), curve_nu=nu.astype(np.float64))
        records["curve"] = {"workload": "100k cluster curve, one pair", "graph": g, "points_sha256": synth.sha256(X),
                            "mu_sha256": synth.sha256(mu), "nu_sha256": synth.sha256(nu), "K": 30, "J": 500,
                            "runs": []}
        jobs += [("job_curve", t) for t in (0.5, 2.0, 8.0)]
    if "bary" in args.which or "grad" in args.which:
        X, labels, H = synth.barycenter_workload()
        log(f"bary: building the oracle graph of {X.shape}")
        L, g = oracle_graph(X, 15, args.procs)
        log(f"bary graph {g}")
        STATE.update(bary_L=L, bary_graph=g, bary_H=H, bary_J=20)
        if "bary" in args.which:
            X2, _, H2 = synth.barycenter_workload(667, 100, 5000)
            L2, g2 = oracle_graph(X2, 15, args.procs)
            log(f"bary20k graph {g2}")
            STATE.update(bary20k_L=L2, bary20k_graph=g2, bary20k_H=H2, bary20k_J=300)
            records["bary"] = {"workload": "200k barycenter (20 iterations) and its 20k twin (300 iterations)",
                               "graph": g, "points_sha256": synth.sha256(X), "H_sha256": synth.sha256(H),
                               "twin_graph": g2, "twin_points_sha256": synth.sha256(X2),
                               "twin_H_sha256": synth.sha256(H2), "K": 40, "t": 2.0, "m": int(H.shape[1])}
            jobs += [("job_bary", "bary"), ("job_bary", "bary20k")]
        if "grad" in args.which:
            mu, nu = synth.gradient_pairs(labels)
            rng = np.random.default_rng(4242)
            spec = []
            for c in range(4):
                supp = np.nonzero(mu[:, c] > 0)[0]
                spec += [(c, int(i)) for i in np.sort(rng.choice(supp, size=4, replace=False))]
            STATE.update(grad_mu=mu, grad_nu=nu, grad_spec=spec)
            records["grad"] = {"workload": "200k gradients, 32 pairs", "graph": g, "points_sha256": synth.sha256(X),
                               "mu_sha256": synth.sha256(mu), "nu_sha256": synth.sha256(nu), "K": 30, "t": 2.0,
                               "J": 200, "ref_pairs": [0, 1, 2, 3], "fd_rel_step": 1e-4, "fd_t_step": 1e-4}
            jobs += [("job_grad_ref", c) for c in range(4)]
            jobs += [("job_grad_fd", (spec[q:q + 4], rel)) for rel in (1e-4, 1e-3) for q in range(0, 16, 4)]
            jobs += [("job_grad_fd_t", c) for c in range(4)]
    if "local1m" in args.which:
        rp, col, w = synth.local_graph_1m()
        n = rp.shape[0] - 1
        L, g = graph_record(n, rp, col, w)
        log(f"local1m graph {g}")
        mu, nu = synth.loguniform_pair_batch(n, 32, 5000, 200000, 10)
        sizes = (mu > 0).sum(axis=0) + (nu > 0).sum(axis=0)
        cols = sorted(int(c) for c in np.argsort(sizes, kind="stable")[:2])
        STATE.update(local1m_L=L, local1m_graph=g, local1m_mu=mu, local1m_nu=nu)
        records["local1m"] = {"workload": "1M random local graph, 32 pairs", "graph": g,
                              "mu_sha256": synth.sha256(mu), "nu_sha256": synth.sha256(nu), "K": 50, "t": 2.0,
                              "J": 200, "ref_pairs": cols}
        jobs += [("job_local1m", c) for c in cols]

    order = ["job_local1m", "job_grad_fd", "job_bary", "job_grad_ref", "job_grad_fd_t", "job_curve"]
    jobs.sort(key=lambda j: order.index(j[0]))   # longest first
    log(f"{len(jobs)} oracle jobs on {args.procs} processes")
    arrays = {k: {} for k in records}
    with mp.get_context("fork").Pool(min(args.procs, len(jobs))) as pool:
        for name, arg, res in pool.imap_unordered(run_job, jobs):
            js, arr = split_arrays(res)
            if name == "job_curve":
                records["curve"]["runs"].append(js)
                arrays["curve"][f"row_t{arg}"] = arr["row_marginal"]
                records["curve"]["runs"].sort(key=lambda r: r["t"])
            elif name == "job_bary":
                key = "full" if arg == "bary" else "twin"
                records["bary"][key] = js
                arrays["bary"][f"p_{key}"] = arr["p"]
            elif name == "job_grad_ref":
                records["grad"][f"ref_{arg}"] = js
                arrays["grad"].update({f"{k}_{arg}": v for k, v in arr.items()})
            elif name == "job_grad_fd":
                records["grad"].setdefault("fd_mu", []).extend(js)
            elif name == "job_grad_fd_t":
                records["grad"][f"fd_t_{arg}"] = js
            elif name == "job_local1m":
                records["local1m"][f"ref_{arg}"] = js
                arrays["local1m"].update({f"{k}_{arg}": v for k, v in arr.items()})
    if "grad" in records:
        rg = records["grad"]
        allfd = rg.pop("fd_mu")
        fd = sorted([r for r in allfd if r["rel"] == 1e-4], key=lambda r: (r["pair"], r["node"]))
        fd3 = {(r["pair"], r["node"]): r for r in allfd if r["rel"] == 1e-3}
        for c in range(4):
            for r, g_ref in zip([r for r in fd if r["pair"] == c], rg[f"ref_{c}"]["dmu_at_fd"]):
                r["ref"] = g_ref
                r["fd_rel1e-3"] = fd3[(r["pair"], r["node"])]["fd"]
                r["h_rel1e-3"] = fd3[(r["pair"], r["node"])]["h"]
                del r["rel"]
        rg["fd_mu"] = fd
        worst_mu = max(abs(r["ref"] - r["fd"]) / abs(r["fd"]) for r in fd)
        worst_mu3 = max(abs(r["ref"] - r["fd_rel1e-3"]) / abs(r["fd_rel1e-3"]) for r in fd)
        worst_t = max(abs(rg[f"ref_{c}"]["dt"] - rg[f"fd_t_{c}"]) / abs(rg[f"fd_t_{c}"]) for c in range(4))
        rg["ref_vs_fd_max_rel"] = {"mu": worst_mu, "mu_rel_step_1e-3": worst_mu3, "t": worst_t}
        log(f"grad: float64 reference vs central differences: mu {worst_mu:.2e} (step 1e-3: {worst_mu3:.2e}), "
            f"t {worst_t:.2e}")
    for name in records:
        save(name, records[name], arrays[name])


if __name__ == "__main__":
    main()

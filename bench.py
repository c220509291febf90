#!/usr/bin/env python3
"""Benchmark: batched forward + backward Geodesic Sinkhorn on a 1M-node kNN graph.

Workload: n = 1M points in R^100 from 50 Gaussian clusters (sigma = 0.1) on a
random 2-D spline surface; symmetrised k = 10 kNN graph with Gaussian-median
weights; heat kernel of degree K = 50 at t = 2; 256 histograms with support
sizes log-uniform in [5k, 200k] (Dirichlet(1) weights on random nodes); the
32,896 pairs i <= j of the 256 x 256 distance matrix are processed in batches
of P pairs; all 256 histograms stay resident in HBM as one n x 256 matrix.
One step = the batch's mu and nu columns gathered from that matrix,
Algorithm 1 for the P pairs (J = 200 iterations) plus the hand-written
reverse sweep giving d D / d mu, d D / d nu
and d D / d t for every pair, whose histogram gradients are then added into
the gradient of the total distance with respect to each of the 256
histograms (256 x n, kept in HBM across steps).  By default the forward records every
iteration's denominators in HBM (51 GB at this size) and the reverse sweep
recomputes nothing; --ckpt-every C > 0 checkpoints w every C iterations
instead and recomputes each segment.

Reported value: heat-kernel applies/s over the timed steps, counting one
single-RHS application per column per Chebyshev chain of the forward pass and
of the adjoint sweep (B * (2J + 2J) per step); recomputation of checkpoint
segments (checkpoint mode only) is extra work, counted separately.  Also reported: the plain
single-RHS form (B = 1) of the same fwd + bwd, the roofline of the fused
Chebyshev step kernel (algorithmic bytes / its HIP-event duration), and the
float64 oracle timed on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "heat-kernel applies/s + HBM GB/s; fwd+bwd batched vs plain, n=1M kNN"
PEAK_HBM_GBS = 8000.0


def method_step_bytes(n: int, nnz: int, B: int, K: int) -> float:
    """Algorithmic bytes of one Chebyshev step launch, averaged over a K-step
    application (forward form, no scaling epilogue), as the method moves them:
    every step streams the CSR and a degree vector once, 4(n+1) + 8 nnz + 4n
    bytes, and five float32 n x B vector passes (the gathered T_{k-1} counted
    once, T_{k-2} read, T_k written, the accumulator read and written), the
    first step three (x read, T_1 and the accumulator written)."""
    csr = 4.0 * (n + 1) + 8.0 * nnz + 4.0 * n
    vec = 4.0 * n * B
    return csr + vec * (3 + 5 * (K - 1)) / K


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--pairs", type=int, default=32, help="pairs per batch (RHS columns)")
    p.add_argument("--iters", type=int, default=200)
    p.add_argument("--K", type=int, default=50)
    p.add_argument("--t", type=float, default=2.0)
    p.add_argument("--ckpt-every", type=int, default=-1,
                   help="checkpoint interval C > 0, or -1: record every iteration (no recomputation)")
    p.add_argument("--per-cluster", type=int, default=20000, help="points per cluster (50 clusters)")
    p.add_argument("--knn", type=int, default=10)
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--ckpt-figure", type=int, default=10,
                   help="with records (the default), also time one step with checkpoints every C iterations "
                        "(0: skip)")
    p.add_argument("--no-other-graphs", action="store_true",
                   help="skip the step kernel's roofline on the banded and torus graphs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the barycenter / plain-forward / Swiss-roll timings")
    p.add_argument("--study", choices=["orders", "footprint", "frontier", "reuse"], default=None,
                   help="instead of the benchmark: the step kernel and its gathers under several node orders, "
                        "the gather rate against the operand's footprint, frontier-sparse steps on and off, "
                        "or the gather reuse an on-chip tile could capture")
    p.add_argument("--probe-only", action="store_true",
                   help="set up the workload, then only time the fused step kernel and the copy kernel "
                        "(short run for profilers and counter collection)")
    return p.parse_args()


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2211_00805_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


TUNE_CACHE = os.path.join(ROOT, "paper_2211_00805_amd", "tune_cache.json")


def shape_key(desc: str) -> str:
    """The launch-shape part of a plan description (vec, S, C, XCD order, CSR hint, ldp)."""
    return " ".join(w for w in desc.split() if w.split("=")[0] in ("vec", "S", "C", "xcd", "csr", "ldp"))


def measured_traffic(shape_desc: str, n: int, nnz: int, B: int):
    """HBM bytes per launch of the step kernel from committed rocprofv3 counter runs.

    Only used when the counters were taken on the current kernel source and
    the same problem shape; otherwise None.
    """
    path = os.path.join(ROOT, "profiles", "cheb_step_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel_sha") != kernel_source_hash() or rec.get("n") != n or rec.get("nnz") != nnz
            or rec.get("B") != B or rec.get("shape") != shape_key(shape_desc)):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(rp, col, w, K: int, t: float, lam: float, mu, nu, csr_sha: str):
    """The float64 oracle on a bounded sample of the workload, on its own graph.

    The oracle takes the benchmark's exported CSR (float32 weights upcast) and
    lambda_hat: one heat application at B = 1 and one at B = 16 (scipy CSR
    products, single thread), and the headline sample, one Sinkhorn iteration
    forward + reverse sweep (gradients in mu, nu and t) for one pair of the
    first batch.  Applies counted as on the GPU: B * (2J + 2J); the single
    applications are reported beside it.
    """
    import numpy as np

    from oracle import graph as ograph
    from oracle import heat
    from oracle import sinkhorn as osk

    n = rp.shape[0] - 1
    L = ograph.laplacian(ograph.csr_from_arrays(n, rp, col, w.astype(np.float64)))
    rng = np.random.default_rng(12)
    single = {}
    for B in (1, 16):
        x = rng.uniform(0.05, 1.0, size=(n, B))
        t0 = time.perf_counter()
        heat.heat_apply(L, lam, t, K, x)
        dt = time.perf_counter() - t0
        single[f"B={B}"] = {"seconds": round(dt, 2), "applies_per_s": round(B / dt, 3)}
    J = 1
    t0 = time.perf_counter()
    osk.sinkhorn_grad(L, lam, t, K, mu[:, :1].astype(np.float64), nu[:, :1].astype(np.float64), J)
    dt = time.perf_counter() - t0
    applies = 1 * (2 * J + 2 * J)
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    parallel = cpu_rhs_parallel(rp, col, w, K, t, lam, min(16, ncores))
    return {"value": applies / dt, "unit": "heat-kernel applies/s", "cores": 1, "kind": "oracle",
            "sample": (f"float64 oracle (scipy CSR products, single thread; host affinity {ncores} cores, "
                       f"os.cpu_count() {os.cpu_count()}) on the workload's own graph (exported CSR sha256 "
                       f"{csr_sha[:16]}, n={n}, nnz={col.shape[0]}, same lambda_hat): 1 Sinkhorn iteration "
                       f"forward + reverse sweep for 1 pair of the first batch, K={K}, t={t}; {applies} applies "
                       f"in {dt:.1f} s"),
            "single_applies": single, "rhs_parallel": parallel}


_RHS_CHILD = r"""
import os, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import graph as ograph
from oracle import heat
d, i, K, t, lam = sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), float(sys.argv[5]), float(sys.argv[6])
rp, col, w = (np.load(os.path.join(d, f + ".npy")) for f in ("rp", "col", "w"))
L = ograph.laplacian(ograph.csr_from_arrays(rp.shape[0] - 1, rp, col, w.astype(np.float64)))
x = np.random.default_rng(100 + i).uniform(0.05, 1.0, size=(rp.shape[0] - 1, 1))
open(os.path.join(d, f"ready{i}"), "w").close()
while not os.path.exists(os.path.join(d, "go")):
    time.sleep(0.01)
t0 = time.perf_counter()
heat.heat_apply(L, lam, t, K, x)
print(time.perf_counter() - t0, flush=True)
"""


def cpu_rhs_parallel(rp, col, w, K: int, t: float, lam: float, procs: int):
    """The oracle's single-RHS heat application in `procs` processes at once (one per host core).

    Each process (a fresh interpreter, one thread) loads the exported CSR,
    builds the float64 Laplacian, waits for a common start, and times one
    application at B = 1; throughput = processes / the slowest one's time.
    """
    import shutil
    import subprocess
    import tempfile

    import numpy as np

    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    d = tempfile.mkdtemp(prefix="gs_cpu_", dir=base)
    try:
        for name, arr in (("rp", rp), ("col", col), ("w", w)):
            np.save(os.path.join(d, name + ".npy"), arr)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        kids = [subprocess.Popen([sys.executable, "-c", _RHS_CHILD, ROOT, d, str(i), str(K), str(t), repr(lam)],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
                for i in range(procs)]
        deadline = time.time() + 300
        while (not all(os.path.exists(os.path.join(d, f"ready{i}")) for i in range(procs))
               and time.time() < deadline and all(k.poll() is None for k in kids)):
            time.sleep(0.05)
        open(os.path.join(d, "go"), "w").close()
        times = []
        for k in kids:
            out, err = k.communicate(timeout=600)
            if k.returncode != 0:
                raise RuntimeError(f"oracle worker failed: {err[-500:]}")
            times.append(float(out.strip().splitlines()[-1]))
    finally:
        shutil.rmtree(d, ignore_errors=True)
    return {"processes": procs, "applies_per_s": round(procs / max(times), 3), "seconds_max": round(max(times), 2),
            "seconds_min": round(min(times), 2),
            "sample": f"{procs} processes (one thread each), one B = 1 application of K = {K} each, started together"}


def roofline_on_other_graphs(gs, synth, np, torch, dev, K: int, B: int):
    """The step kernel on 1M-node graphs whose gathers can hit cache, in its autotuned launch.

    band_matched_nnz: each node draws 9 partners within +-20,000 ids (18.0M
    nonzeros, the kNN graph's size); band_narrow: within +-2,000 ids; torus:
    the 1000 x 1000 torus (4 nonzeros per row).  Same algorithmic byte count
    and peak as the headline roofline.
    """
    out = {}
    graphs = {"band_matched_nnz": lambda: synth.random_local_graph(1_000_000, 9, 20000, np.random.default_rng(91)),
              "band_narrow": lambda: synth.random_local_graph(1_000_000, 9, 2000, np.random.default_rng(92)),
              "torus_1000x1000": lambda: synth.torus_graph(1000, 1000)}
    for name, make in graphs.items():
        arrs = make()
        n = arrs[0].shape[0] - 1
        g = gs.gs_graph_from_csr(n, *arrs)
        plan = gs.Plan(g, K, B, flags=gs.GS_PLAN_AUTOTUNE)
        ms, _ = gs.gs_plan_time_step(plan, reps=4)
        alg = method_step_bytes(n, g.nnz, B, K)
        out[name] = {"n": n, "nnz": g.nnz, "us": round(ms * 1e3, 1), "achieved_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
                     "frac": round(alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), "plan": plan.describe()}
        log(f"[roofline] {name}: {ms * 1e3:.1f} us, frac {out[name]['frac']:.3f}")
        del plan, g
    return out


def extra_workloads(gs, synth, np, torch, dev):
    """Timings of the other paper-shaped workloads (one run each after a warm run).

    barycenter: n ~ 200k (30 clusters x 6667 on a curve in R^50, k = 15), m = 64
      inputs with log-uniform [1k, 50k] supports and Dirichlet(0.5) weights,
      alpha = 1/64, K = 40, t = 2, J = 300, all inputs in one multi-RHS launch.
    gradient: the same graph, 32 pairs of Dirichlet(1) histograms on adjacent
      blocks of 3 clusters (~20k nodes each, random start), K = 30, t = 2,
      J = 200: forward with records + reverse sweep (mu, nu and t).
    plain_forward: n = 100k (20 clusters x 5000, R^50, k = 15), one pair with
      Dirichlet(1) on clusters 0-3 vs 4-7, K = 30, J = 500, t in {0.5, 2, 8}.
    swiss_roll: n = 2000 Swiss roll in R^10, k = 10, K = 20, t = 1, uniform
      histograms on 500 random nodes, J = 200.
    swiss_roll_nn: 15 Gaussians x 10,000 samples on a Swiss roll rotated into
      R^10 (n = 150k, k = 10), all 105 pairs, K = 50, t = 2, J = 200; graph
      time and distance time, scores against intrinsic-coordinate ground truth;
      the same pairs with the backward-Euler kernel (N = 10 implicit steps,
      CG to the automatic iteration count), the paper's comparator.
    barycenter_effect: control 10 x N(0, 1), treatment 9 x N(5, 1) + one at
      -30, 500 samples each in 1-D (k = 10), K = 30, t = 2, J = 100; two
      barycenters and the effect.
    """
    out = {}
    # barycenter
    X, labels3 = synth.clusters_on_curve(30, 6667, dim=50, sigma=0.1, workload=3)
    g = gs.gs_graph_from_points(X, 15)
    lam = gs.gs_lambda_max(g, iters=60, seed=3, safety=1.01)
    m, K, t, J = 64, 40, 2.0, 300
    rng = np.random.default_rng(synth.seed_for(3, 2))
    H, _ = synth.loguniform_support_histograms(g.n, m, 1000, 50000, 0.5, rng)
    Hd = torch.from_numpy(H).to(dev)
    plan = gs.Plan(g, K, m, flags=gs.GS_PLAN_AUTOTUNE)
    bary = torch.empty(g.n, device=dev)
    alpha = np.full(m, 1.0 / m)
    gs.gs_barycenter(plan, lam, t, Hd, alpha, 2, bary)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    gs.gs_barycenter(plan, lam, t, Hd, alpha, J, bary)
    torch.cuda.synchronize()
    dt = time.perf_counter() - w0
    out["barycenter"] = {"n": g.n, "nnz": g.nnz, "m": m, "K": K, "iters": J, "seconds": round(dt, 3),
                         "iterations_per_s": round(J / dt, 1), "applies_per_s": round(2 * m * J / dt, 1),
                         "plan": plan.describe(), "mass": round(float(bary.sum().item()), 6)}
    log(f"[extra] barycenter {dt:.2f}s")
    del plan, Hd
    # differentiation on the same graph: 32 pairs on adjacent blocks of 3 clusters (~20k nodes), K = 30,
    # t = 2, J = 200, forward recording every iteration + reverse sweep (gradients in mu, nu and t)
    B4, K4, J4 = 32, 30, 200
    rng = np.random.default_rng(synth.seed_for(4, 2))
    pairs = [synth.cluster_block_pair(labels3, int(rng.integers(0, 24)), 3, 1.0, rng) for _ in range(B4)]
    mu4 = torch.from_numpy(np.stack([p_[0] for p_ in pairs], axis=1)).to(dev)
    nu4 = torch.from_numpy(np.stack([p_[1] for p_ in pairs], axis=1)).to(dev)
    plan4 = gs.Plan(g, K4, B4, flags=gs.GS_PLAN_AUTOTUNE)
    rec4 = torch.empty(gs.ckpt_floats(plan4, J4, gs.GS_RECORD_ALL), device=dev)
    gmu4 = torch.empty(g.n * B4, device=dev)
    gnu4 = torch.empty(g.n * B4, device=dev)

    def grad_step(J_):
        gs.gs_sinkhorn(plan4, lam, 2.0, mu4, nu4, J_, ckpt_every=gs.GS_RECORD_ALL, ckpt=rec4)
        return gs.gs_sinkhorn_backward(plan4, lam, 2.0, mu4, nu4, J_, gs.GS_RECORD_ALL, rec4, np.ones(B4),
                                       grad_mu=gmu4, grad_nu=gnu4)

    grad_step(2)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    gt4 = grad_step(J4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - w0
    out["gradient"] = {"n": g.n, "nnz": g.nnz, "pairs": B4, "K": K4, "iters": J4, "seconds": round(dt, 3),
                       "applies_per_s": round(4 * J4 * B4 / dt, 1), "plan": plan4.describe(),
                       "grad_t_finite": bool(np.all(np.isfinite(gt4)))}
    log(f"[extra] gradient fwd+bwd {dt:.2f}s")
    del plan4, rec4, gmu4, gnu4, g
    # plain forward on the cluster-curve graph
    X, labels = synth.clusters_on_curve(20, 5000, dim=50, sigma=0.1, workload=2)
    g = gs.gs_graph_from_points(X, 15)
    lam = gs.gs_lambda_max(g, iters=60, seed=2, safety=1.01)
    mu, nu = synth.cluster_block_pair(labels, 0, 4, 1.0, np.random.default_rng(synth.seed_for(2, 2)))
    mud, nud = torch.from_numpy(mu).to(dev), torch.from_numpy(nu).to(dev)
    plan = gs.Plan(g, 30, 1, flags=gs.GS_PLAN_AUTOTUNE)
    pf = {"n": g.n, "nnz": g.nnz, "K": 30, "iters": 500, "plan": plan.describe()}
    for t in (0.5, 2.0, 8.0):
        gs.gs_sinkhorn(plan, lam, t, mud, nud, 2)
        w0 = time.perf_counter()
        r = gs.gs_sinkhorn(plan, lam, t, mud, nud, 500)
        dt = time.perf_counter() - w0
        pf[f"t={t}"] = {"ms": round(dt * 1e3, 2), "applies_per_s": round(1000 / dt, 1), "D": float(r["dist"][0])}
    out["plain_forward"] = pf
    log("[extra] plain forward done")
    del plan, g
    # Swiss roll
    X = synth.swiss_roll(2000, 10, 0.05, workload=1)
    g = gs.gs_graph_from_points(X, 10)
    lam = gs.gs_lambda_max(g, iters=60, seed=1, safety=1.01)
    rng = np.random.default_rng(synth.seed_for(1, 2))
    mu = torch.from_numpy(synth.uniform_on_random_nodes(2000, 500, rng)).to(dev)
    nu = torch.from_numpy(synth.uniform_on_random_nodes(2000, 500, rng)).to(dev)
    plan = gs.Plan(g, 20, 1, flags=gs.GS_PLAN_AUTOTUNE)
    gs.gs_sinkhorn(plan, lam, 1.0, mu, nu, 2)
    w0 = time.perf_counter()
    r = gs.gs_sinkhorn(plan, lam, 1.0, mu, nu, 200)
    dt = time.perf_counter() - w0
    out["swiss_roll"] = {"n": 2000, "nnz": g.nnz, "K": 20, "iters": 200, "ms": round(dt * 1e3, 2),
                         "launches_per_s": round(2 * 20 * 200 / dt, 0), "D": float(r["dist"][0])}
    log("[extra] swiss roll done")
    del plan, g
    # nearest-Wasserstein-neighbour experiment on the Swiss roll
    per = 10000
    X, lab, means = synth.gaussians_on_swiss_roll(15, per)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    g = gs.gs_graph_from_points(X, 10)
    lam = gs.gs_lambda_max(g, iters=60, seed=5, safety=1.01)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - w0
    H = np.zeros((g.n, 15), dtype=np.float32)
    for i in range(15):
        H[lab == i, i] = 1.0 / per
    Hd = torch.from_numpy(H).to(dev)
    gs.distance_matrix(g, lam, 2.0, 50, Hd[:, :3], 2)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    D = gs.distance_matrix(g, lam, 2.0, 50, Hd, 200)
    torch.cuda.synchronize()
    t_dist = time.perf_counter() - w0
    truth = np.linalg.norm(means[:, None] - means[None], axis=2)
    sc = {k: round(v, 4) for k, v in gs.nn_scores(D, truth).items()}
    out["swiss_roll_nn"] = {"n": g.n, "nnz": g.nnz, "pairs": 105, "K": 50, "t": 2.0, "iters": 200,
                            "graph_seconds": round(t_graph, 3), "distance_seconds": round(t_dist, 3),
                            "total_seconds": round(t_graph + t_dist, 3), "scores": sc}
    log(f"[extra] swiss roll nn {t_graph:.2f}s + {t_dist:.2f}s {sc}")
    eplan = gs.Plan(g, 50, 32)
    eplan.set_kernel(gs.GS_KERNEL_EULER, 10)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    De = gs.distance_matrix(g, lam, 2.0, 50, Hd, 200, plan=eplan)
    torch.cuda.synchronize()
    t_euler = time.perf_counter() - w0
    sce = {k: round(v, 4) for k, v in gs.nn_scores(De, truth).items()}
    out["swiss_roll_nn"]["euler"] = {"N": 10, "plan": eplan.describe(), "distance_seconds": round(t_euler, 3),
                                     "scores": sce, "time_ratio_vs_chebyshev": round(t_euler / t_dist, 2)}
    log(f"[extra] swiss roll nn euler {t_euler:.2f}s {sce}")
    del g, Hd, eplan
    # Expected Barycenter Effect with an outlier at -30
    rng = np.random.default_rng(12)
    control = [rng.normal(0.0, 1.0, 500) for _ in range(10)]
    treat = [rng.normal(5.0, 1.0, 500) for _ in range(9)] + [rng.normal(-30.0, 1.0, 500)]
    pts = np.concatenate(control + treat).astype(np.float32)[:, None]
    Hf = np.zeros((pts.shape[0], 20), dtype=np.float32)
    for i in range(20):
        Hf[i * 500:(i + 1) * 500, i] = 1.0 / 500
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    g = gs.gs_graph_from_points(pts, 10)
    lam = gs.gs_lambda_max(g, iters=60, seed=3, safety=1.01)
    Hfd = torch.from_numpy(Hf).to(dev)
    alpha = np.full(10, 0.1)
    pT = gs.family_barycenter(g, lam, 2.0, 30, Hfd[:, 10:].contiguous(), alpha, 100)
    pC = gs.family_barycenter(g, lam, 2.0, 30, Hfd[:, :10].contiguous(), alpha, 100)
    tau = float(gs.expected_barycenter_effect(pT, pC, torch.from_numpy(pts).to(dev))[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - w0
    naive = float(np.mean(np.concatenate(treat)) - np.mean(np.concatenate(control)))
    out["barycenter_effect"] = {"n": g.n, "outlier": -30.0, "K": 30, "iters": 100, "seconds": round(dt, 3),
                                "effect": round(tau, 4), "naive_difference_of_means": round(naive, 4)}
    log(f"[extra] barycenter effect {tau:.4f} (naive {naive:.4f}) {dt:.2f}s")
    return out


def node_orders(X, labels, rp, col, np):
    """Node orders of the 1M workload compared by the order study (new id -> old id).

    generator: cluster after cluster (the generator's own order); random: a
    uniform permutation; cluster_grid: the clusters of the 10 x 5 parameter grid
    renumbered column-major, so grid neighbours (the clusters a node's kNN
    edges mostly reach) are adjacent; rcm: reverse Cuthill-McKee of the graph;
    pca: sorted by the first principal component; pca_bisect: recursive
    bisection at the median of each part's own first principal component down
    to parts of <= 4096 nodes (a geometric partition order).
    """
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    n = X.shape[0]
    out = {"generator": np.arange(n), "random": np.random.default_rng(7).permutation(n)}
    grid = np.arange(50).reshape(10, 5)
    cl_order = grid.T.ravel()                      # column-major walk of the 10 x 5 grid
    out["cluster_grid"] = np.concatenate([np.nonzero(labels == c)[0] for c in cl_order])
    A = csr_matrix((np.ones(col.shape[0], dtype=np.float32), col, rp), shape=(n, n))
    out["rcm"] = np.asarray(reverse_cuthill_mckee(A, symmetric_mode=True), dtype=np.int64)

    def top_pc(Y):
        Yc = Y - Y.mean(axis=0)
        v = np.random.default_rng(0).standard_normal(Y.shape[1])
        for _ in range(8):
            v = Yc.T @ (Yc @ v)
            v /= np.linalg.norm(v)
        return Yc @ v

    out["pca"] = np.argsort(top_pc(X), kind="stable")
    parts = [np.arange(n)]
    while max(len(p) for p in parts) > 4096:
        nxt = []
        for p in parts:
            if len(p) <= 4096:
                nxt.append(p)
                continue
            o = np.argsort(top_pc(X[p]), kind="stable")
            h = len(p) // 2
            nxt += [p[o[:h]], p[o[h:]]]
        parts = nxt
    out["pca_bisect"] = np.concatenate(parts)
    return out


def permuted_csr(rp, col, w, order, np):
    """CSR of the graph renumbered so that new node i is old node order[i] (rows sorted by column)."""
    n = rp.shape[0] - 1
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    deg = np.diff(rp)[order]
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(deg)
    src = np.repeat(np.arange(n), deg)
    starts = rp[order]
    e_old = starts[src] + (np.arange(rp2[-1]) - rp2[src])
    c2 = inv[col[e_old]]
    w2 = w[e_old]
    key = src * n + c2
    o = np.argsort(key, kind="stable")
    return rp2.astype(np.int32), c2[o].astype(np.int32), w2[o].astype(np.float32)


def reuse_study(args):
    """How much gather reuse any on-chip tile could capture (one JSON line).

    For parts of P consecutive rows of the 1M workload under four node orders,
    the rows a part gathers from: distinct(neighbours) / nonzeros is the
    share of the gathers that remain even if a cache or an LDS tile held
    every row the part needs, and distinct x 128 B is the capacity that would
    take (B = 32 float columns).  P = 16 is one block of the benchmark's
    launch shape, 256 and 1024 what an LDS tile could cover, 32768 about one
    4 MB L2 of 128-byte rows, 125000 one XCD's row range under the XCD-aware
    block order.
    """
    import numpy as np

    import paper_2211_00805_amd as gs
    import synth

    X, labels = synth.clusters_on_surface((10, 5), args.per_cluster, 100, 0.1, workload=5)
    g0 = gs.gs_graph_from_points(X, args.knn)
    rp, col, w, _ = g0.export()
    del g0
    log("[study] computing node orders ...")
    orders = node_orders(X, labels, rp, col, np)
    del X
    n, nnz = int(rp.shape[0] - 1), int(col.shape[0])
    res = {"study": "gather reuse", "n": n, "nnz": nnz, "row_bytes": 128, "orders": {}}
    for name in ("generator", "cluster_grid", "pca_bisect", "random"):
        rp2, c2, _ = permuted_csr(rp, col, w, orders[name], np)
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp2))
        per = {}
        for P in (16, 256, 1024, 32768, 125000):
            distinct = int(np.unique((rows // P) * n + c2.astype(np.int64)).size)
            nparts = (n + P - 1) // P
            per[str(P)] = {"distinct_over_nnz": round(distinct / nnz, 4),
                           "mean_working_set_kb": round(distinct / nparts * 128 / 1024, 1)}
        res["orders"][name] = per
        log(f"[study] {name}: {per}")
    print(json.dumps(res), flush=True)


def order_study(args):
    """The step kernel and its gathers alone under each node order of the 1M workload (one JSON line)."""
    import numpy as np
    import torch

    import paper_2211_00805_amd as gs
    import synth

    dev = torch.device("cuda:0")
    X, labels = synth.clusters_on_surface((10, 5), args.per_cluster, 100, 0.1, workload=5)
    g0 = gs.gs_graph_from_points(X, args.knn)
    rp, col, w, _ = g0.export()
    del g0
    log("[study] computing node orders ...")
    orders = node_orders(X, labels, rp, col, np)
    del X
    K, B = args.K, 32
    res = {"study": "node orders", "n": int(rp.shape[0] - 1), "nnz": int(col.shape[0]), "K": K, "B": B,
           "shape": "vec=4 S=2 C=8 xcd=1", "orders": {}}
    for name, order in orders.items():
        rp2, c2, w2 = permuted_csr(rp, col, w, order, np)
        n = rp2.shape[0] - 1
        rows = np.repeat(np.arange(n), np.diff(rp2))
        d = np.abs(rows - c2.astype(np.int64))
        g = gs.gs_graph_from_csr(n, rp2, c2, w2)
        plan = gs.Plan(g, K, B)
        plan.set_shape(4, 2, 8)
        step_ms, _ = gs.gs_plan_time_step(plan, reps=4)
        idx = torch.from_numpy(c2).to(dev)
        Xop = torch.ones((n, 32), device=dev)
        gout = torch.empty((len(c2) + 31) // 32 * 32, device=dev)
        for _ in range(2):
            gs.gs_stream_gather(Xop, idx, gout)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            gs.gs_stream_gather(Xop, idx, gout)
        e1.record()
        torch.cuda.synchronize()
        gather_us = e0.elapsed_time(e1) * 1e3 / 5
        alg = method_step_bytes(n, len(c2), B, K)
        res["orders"][name] = {"step_us": round(step_ms * 1e3, 1), "gather_us": round(gather_us, 1),
                               "frac": round(alg / (step_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                               "median_abs_i_minus_j": float(np.median(d)),
                               "within_16k": round(float(np.mean(d < 16384)), 4),
                               "within_128k": round(float(np.mean(d < 131072)), 4)}
        log(f"[study] {name}: {res['orders'][name]}")
        del plan, g, idx, Xop, gout
    print(json.dumps(res), flush=True)


def footprint_study(args):
    """Gather rate against the gathered operand's footprint (one JSON line).

    The step kernel's gather path alone (gs_stream_gather: one 128-byte row of
    an rows x 32 float32 operand per index, 18,322,390 indices as the 1M kNN
    graph has nonzeros): uniform random indices over operands from 1 MB
    (inside one XCD's 4 MB L2) through 128 MB (the 1M operand; inside the
    256 MB Infinity Cache) to 2 GB (HBM only); and indices within +-W rows of a
    ramp over a 1M-row operand (banded locality).
    """
    import torch

    import paper_2211_00805_amd as gs

    dev = torch.device("cuda:0")
    m = 18322390
    gen = torch.Generator(device=dev)
    gen.manual_seed(1)
    out = torch.empty((m + 31) // 32 * 32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def gather_us(Xop, idx, reps=5):
        gs.gs_stream_gather(Xop, idx, out)
        e0.record()
        for _ in range(reps):
            gs.gs_stream_gather(Xop, idx, out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    res = {"study": "gather footprint", "indices": m, "row_bytes": 128, "uniform": {}, "band_1M_rows": {}}
    for rows in [8192, 16384, 32768, 65536, 131072, 262144, 524288, 1 << 20, 2 << 20, 4 << 20, 8 << 20, 16 << 20]:
        Xop = torch.ones((rows, 32), device=dev)
        idx = torch.randint(0, rows, (m,), device=dev, dtype=torch.int32, generator=gen)
        us = gather_us(Xop, idx)
        res["uniform"][str(rows)] = {"MB": round(rows * 128 / 1e6, 1), "us": round(us, 1),
                                     "gbs": round(m * 128 / us / 1e3, 1)}
        log(f"[study] uniform over {rows} rows: {res['uniform'][str(rows)]}")
        del Xop, idx
    n = 1 << 20
    Xop = torch.ones((n, 32), device=dev)
    ramp = torch.arange(m, device=dev, dtype=torch.int64) * n // m
    for W in [512, 2048, 8192, 32768, 131072, 524288]:
        off = torch.randint(-W, W + 1, (m,), device=dev, generator=gen)
        idx = ((ramp + off) % n).to(torch.int32)
        us = gather_us(Xop, idx)
        res["band_1M_rows"][str(W)] = {"us": round(us, 1), "gbs": round(m * 128 / us / 1e3, 1)}
        log(f"[study] band +-{W}: {res['band_1M_rows'][str(W)]}")
    print(json.dumps(res), flush=True)


def frontier_study(args):
    """Work a frontier-sparse step could skip, per workload, and what the
    frontier option gains on the GPU (one JSON line).

    T_k of an application is zero outside the k-hop neighbourhood N^k(S) of the
    applied vector's support S (the union over the B columns of a launch, since
    a row is skipped only when all its columns are zero), so step k could skip
    the rows outside N^k(S), at most.  Reported: the fraction of rows and of
    nonzeros (the gathers) inside N^k(S) for k = 0..4, and the largest share
    of an application's gathers a frontier-sparse kernel could skip,
    sum_k (1 - nnz(N^{k-1}(S)) / nnz) / K (step k gathers T_{k-1}).  Measured:
    gs_heat_apply (and gs_sinkhorn, J = 6, where the workload has pairs) on a
    plan with the frontier option and one without, calls interleaved, the
    level computation included, and whether the two agree bit for bit.
    """
    import numpy as np
    import scipy.sparse as sp

    import paper_2211_00805_amd as gs
    import synth

    def reach(rp, col, S, K):
        n = rp.shape[0] - 1
        A = sp.csr_matrix((np.ones(col.shape[0], dtype=np.float32), col, rp), shape=(n, n))
        deg = np.diff(rp).astype(np.float64)
        f = S.copy()
        rows, nnzs = [], []
        for k in range(K):
            rows.append(float(f.mean()))
            nnzs.append(float(deg[f].sum() / deg.sum()))
            if k < K - 1:
                f = f | (A @ f.astype(np.float32) > 0)
        skip = float(np.sum(1.0 - np.asarray(nnzs)) / K)   # step k gathers T_{k-1}: hops 0..K-1
        return {"rows_reached": [round(x, 4) for x in rows[:5]], "nnz_reached": [round(x, 4) for x in nnzs[:5]],
                "max_skippable_gather_share": round(skip, 4)}

    import torch

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()

    def measured(g, K, H, pair=None, J=6, t=2.0, rounds=15):
        """Milliseconds of gs_heat_apply on H (and of gs_sinkhorn on pair, J
        iterations) on a plan with the frontier option off and one with it
        on, the calls interleaved round by round (medians), the results
        compared bit for bit."""
        Hd = dev(H)
        B = H.shape[1]
        lam = g.edge_bound
        plans = (gs.Plan(g, K, B), gs.Plan(g, K, B))
        plans[1].set_frontier(1)
        Ys = [torch.empty(H.size, device="cuda") for _ in plans]
        pd = None if pair is None else (dev(pair[0]), dev(pair[1]))
        dist = [None, None]

        def call(i, what):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if what == "heat":
                gs.gs_heat_apply(plans[i], lam, t, Hd, Ys[i])
            else:
                dist[i] = gs.gs_sinkhorn(plans[i], lam, t, pd[0], pd[1], J)["dist"]
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3

        whats = ["heat"] + (["sinkhorn"] if pair is not None else [])
        for w in whats:
            for i in (0, 1):
                call(i, w)
        ts = {(w, i): [] for w in whats for i in (0, 1)}
        for _ in range(rounds):
            for w in whats:
                for i in (0, 1):
                    ts[(w, i)].append(call(i, w))
        out = {}
        for w in whats:
            name = "heat" if w == "heat" else f"sinkhorn_J{J}"
            off, on = float(np.median(ts[(w, 0)])), float(np.median(ts[(w, 1)]))
            out[f"{name}_ms_frontier_off"] = round(off, 3)
            out[f"{name}_ms_frontier_on"] = round(on, 3)
            out[f"{name}_on_over_off"] = round(on / off, 3)
        out["heat_bitwise_equal"] = bool(torch.equal(Ys[0].view(torch.int32), Ys[1].view(torch.int32)))
        if pair is not None:
            out["sinkhorn_bitwise_equal"] = bool(np.array_equal(dist[0], dist[1]))
        for p in plans:
            p.destroy()
        return out

    res = {"study": "frontier", "workloads": {}}
    X, labels, mu, nu = synth.curve_pair_workload()
    g = gs.gs_graph_from_points(X, 15)
    rp, col, _, _ = g.export()
    key = "100k curve, one pair (mu on clusters 0-3), K = 30"
    res["workloads"][key] = reach(rp, col, mu > 0, 30)
    res["workloads"][key].update(measured(g, 30, mu[:, None], pair=(mu[:, None], nu[:, None])))
    X, labels, _ = synth.barycenter_workload()
    g = gs.gs_graph_from_points(X, 15)
    rp, col, _, _ = g.export()
    gm, gn = synth.gradient_pairs(labels)
    key = "200k gradients, 32 pairs (union of the mu supports), K = 30"
    res["workloads"][key] = reach(rp, col, (gm > 0).any(axis=1), 30)
    res["workloads"][key].update(measured(g, 30, gm, pair=(gm, gn), rounds=6))
    key = "200k gradients, pair 0 alone, K = 30"
    res["workloads"][key] = reach(rp, col, gm[:, 0] > 0, 30)
    res["workloads"][key].update(measured(g, 30, gm[:, :1], pair=(gm[:, :1], gn[:, :1])))
    X, labels = synth.clusters_on_surface((10, 5), args.per_cluster, 100, 0.1, workload=5)
    g = gs.gs_graph_from_points(X, args.knn)
    rp, col, _, _ = g.export()
    n = rp.shape[0] - 1
    sizes = synth.loguniform_support_sizes(n, 256, 5000, 200000, synth.seed_for(5, 2))
    H = np.zeros((n, 32), dtype=np.float32)
    for i in range(32):
        H[:, i] = synth.histogram_on_random_support(n, int(sizes[i]), 1.0, synth.seed_for(5, 2) * 1000 + i)
    key = "1M kNN, a batch of 32 random supports, K = 50"
    res["workloads"][key] = reach(rp, col, (H > 0).any(axis=1), 50)
    res["workloads"][key].update(measured(g, 50, H, rounds=5))
    nc = 1_000_000
    gc = gs.gs_graph_from_csr(nc, *synth.cycle_graph(nc))
    Hc = np.zeros((nc, 1), dtype=np.float32)
    Hc[nc // 2, 0] = 1.0
    Hc2 = np.zeros((nc, 1), dtype=np.float32)
    Hc2[nc // 2 + 20, 0] = 1.0
    res["workloads"]["1M cycle, one node each (20 hops apart), K = 50"] = measured(gc, 50, Hc, pair=(Hc, Hc2))
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): only the one-GPU path is built; "
              "the method would shard by pairs (each GPU a share of the pair batches on a full graph replica, "
              "one all-reduce of the histogram gradients at the end).", file=sys.stderr)
        sys.exit(2)

    if args.study == "orders":
        order_study(args)
        return
    if args.study == "footprint":
        footprint_study(args)
        return
    if args.study == "frontier":
        frontier_study(args)
        return
    if args.study == "reuse":
        reuse_study(args)
        return

    import numpy as np
    import torch

    import paper_2211_00805_amd as gs
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, t, J, ce, P = args.K, args.t, args.iters, args.ckpt_every, args.pairs

    # ---------------------------------------------------------------- setup (untimed)
    t0 = time.perf_counter()
    X, labels = synth.clusters_on_surface((10, 5), args.per_cluster, 100, 0.1, workload=5)
    n = X.shape[0]
    log(f"[setup] points {X.shape} in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    g = gs.gs_graph_from_points(X, args.knn)
    t_graph = time.perf_counter() - t0
    log(f"[setup] kNN graph n={g.n} nnz={g.nnz} components={g.n_components} in {t_graph:.1f}s")
    inputs = {"points_sha256": synth.sha256(X)}
    del X
    lam = gs.gs_lambda_max(g, iters=60, seed=5, safety=1.01)
    log(f"[setup] lambda_hat={lam:.4f} (edge bound {g.edge_bound:.4f})")

    m = 256
    sizes = synth.loguniform_support_sizes(n, m, 5000, 200000, synth.seed_for(5, 2))
    pairs = np.array([(i, j) for i in range(m) for j in range(i, m)], dtype=np.int64)
    order = np.random.default_rng(synth.seed_for(5, 3)).permutation(len(pairs))
    nbatch = args.warmup + args.steps
    batches = [pairs[order[b * P:(b + 1) * P]] for b in range(nbatch)]
    t0 = time.perf_counter()
    # all m histograms resident in HBM as one node-major n x m matrix (1 GB); each
    # step gathers its batch's mu and nu columns from it with the library's kernel
    Ht = np.empty((m, n), dtype=np.float32)
    hh = hashlib.sha256()
    for i in range(m):
        Ht[i] = synth.histogram_on_random_support(n, int(sizes[i]), 1.0, synth.seed_for(5, 2) * 1000 + i)
        hh.update(synth.sha256(Ht[i]).encode())
    Hdev = torch.from_numpy(np.ascontiguousarray(Ht.T)).to(dev)
    del Ht
    rp_, col_, w_, _ = g.export()
    inputs.update({"csr_sha256": hashlib.sha256(synth.sha256(rp_).encode() + synth.sha256(col_).encode()
                                                 + synth.sha256(w_).encode()).hexdigest(),
                   "histograms_sha256": hh.hexdigest(), "histograms": m,
                   "seeds": {"points": synth.seed_for(5, 0), "surface": synth.seed_for(5, 1),
                             "support_sizes": synth.seed_for(5, 2), "pair_order": synth.seed_for(5, 3),
                             "histogram_i": f"{synth.seed_for(5, 2)} * 1000 + i", "lambda_max": 5}})
    del rp_, col_, w_
    dev_batches = [(torch.from_numpy(b[:, 0].astype(np.int32)).to(dev),
                    torch.from_numpy(b[:, 1].astype(np.int32)).to(dev)) for b in batches]
    mu = torch.empty((n, P), dtype=torch.float32, device=dev)
    nu = torch.empty_like(mu)
    gs.gs_gather_columns(Hdev, dev_batches[0][0], mu)   # a representative batch for the probes below
    gs.gs_gather_columns(Hdev, dev_batches[0][1], nu)
    log(f"[setup] {m} histograms, {nbatch} batches of {P} pairs in {time.perf_counter() - t0:.1f}s")

    plan = gs.Plan(g, K, P, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE_CACHE)
    shape = plan.describe()
    log(f"[setup] plan: {shape}")
    if args.probe_only:
        step_ms, step_bytes = gs.gs_plan_time_step(plan, reps=2)
        plan.set_kernel(gs.GS_KERNEL_CLENSHAW)
        clen_ms, _ = gs.gs_plan_time_step(plan, reps=2)
        plan.set_kernel(gs.GS_KERNEL_CHEBYSHEV)
        nb = 1 << 30
        src = torch.ones(nb // 4, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            gs.gs_stream_copy(src, dst)
        del src, dst
        gather_us = None
        if P == 32:   # the step kernel's gathers alone (one 128-byte row per nonzero), 3 passes
            _, col, _, _ = g.export()
            idx = torch.from_numpy(col.astype(np.int32)).to(dev)
            gout = torch.empty((len(col) + 31) // 32 * 32, device=dev)
            Xop = mu.view(n, 32)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(3):
                gs.gs_stream_gather(Xop, idx, gout)
            ev1.record()
            torch.cuda.synchronize()
            gather_us = ev0.elapsed_time(ev1) * 1e3 / 3
        torch.cuda.synchronize()
        print(json.dumps({"probe": "2 applications (K step launches each), 2 in Clenshaw's form + copy of 1 GiB x3 "
                                   "+ 3 gather passes",
                          "step_ms": step_ms, "clenshaw_step_ms": clen_ms, "gather_us": gather_us,
                          "step_kernel_bytes": step_bytes, "step_algorithmic_bytes": method_step_bytes(n, g.nnz, P, K),
                          "copy_bytes_read": nb, "copy_bytes_written": nb,
                          "plan": shape, "shape": shape_key(shape), "kernel_sha": kernel_source_hash(),
                          "n": n, "nnz": g.nnz, "B": P, "K": K}), flush=True)
        return
    ckpt = torch.empty(gs.ckpt_floats(plan, J, ce), device=dev)
    log(f"[setup] {'records' if ce == gs.GS_RECORD_ALL else 'checkpoints'}: {ckpt.numel() * 4 / 1e9:.1f} GB")
    gmu = torch.empty(n * P, device=dev)
    gnu = torch.empty(n * P, device=dev)
    ones = np.ones(P)

    # gradient of the total distance with respect to every one of the m histograms
    # (m x n, distribution-major), summed over the batches' pairs
    G = torch.zeros((m, n), dtype=torch.float32, device=dev)
    log(f"[setup] per-histogram gradients: {G.numel() * 4 / 1e9:.1f} GB")

    def step(ci, cj):
        gs.gs_gather_columns(Hdev, ci, mu)
        gs.gs_gather_columns(Hdev, cj, nu)
        out = gs.gs_sinkhorn(plan, lam, t, mu, nu, J, ckpt_every=ce, ckpt=ckpt)
        gt = gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, ce, ckpt, ones, grad_mu=gmu, grad_nu=gnu)
        gs.gs_accumulate_columns(gmu.view(n, P), ci, G)
        gs.gs_accumulate_columns(gnu.view(n, P), cj, G)
        return out["dist"], gt

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step(*dev_batches[w])
        torch.cuda.synchronize()
        log(f"[warmup] step {w} {time.perf_counter() - t0:.2f}s")

    # ---------------------------------------------------------------- timed region
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record()
    dists = []
    for s in range(args.steps):
        d, gt = step(*dev_batches[args.warmup + s])
        dists.append(d)
        log(f"[timed] step {s} done ({time.perf_counter() - wall0:.2f}s), D[0]={d[0]:.6f} dD/dt[0]={gt[0]:.6f}")
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = max(ms_total, wall * 1e3) / args.steps
    applies_per_step = P * (2 * J + 2 * J)
    value = applies_per_step / (ms_per_step / 1e3)
    finite = all(np.all(np.isfinite(d)) for d in dists) and bool(torch.isfinite(G).all())

    # ---------------------------------------------------------------- checkpointed form (one step)
    ckpt_fig = None
    if ce == gs.GS_RECORD_ALL and args.ckpt_figure > 0:
        C = args.ckpt_figure
        ck = torch.empty(gs.ckpt_floats(plan, J, C), device=dev)

        def step_ck(ci, cj):
            gs.gs_gather_columns(Hdev, ci, mu)
            gs.gs_gather_columns(Hdev, cj, nu)
            gs.gs_sinkhorn(plan, lam, t, mu, nu, J, ckpt_every=C, ckpt=ck)
            gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, C, ck, ones, grad_mu=gmu, grad_nu=gnu)

        torch.cuda.synchronize()
        w0 = time.perf_counter()
        step_ck(*dev_batches[args.warmup])
        torch.cuda.synchronize()
        tck = time.perf_counter() - w0
        seg_gb = 2 * C * n * P * 4 / 1e9
        ckpt_fig = {"ckpt_every": C, "ms_per_step": round(tck * 1e3, 1),
                    "value": round(applies_per_step / tck, 1), "unit": "heat-kernel applies/s",
                    "recompute_applies_per_step": P * 2 * J,
                    "hbm_gb": {"checkpoints": round(ck.numel() * 4 / 1e9, 2), "segment_slots": round(seg_gb, 2),
                               "records_instead": round(ckpt.numel() * 4 / 1e9, 2)}}
        log(f"[ckpt] checkpoints every {C}: {tck:.2f}s per step -> {applies_per_step / tck:.0f} applies/s")
        del ck

    # ---------------------------------------------------------------- fused step roofline (HIP events)
    # achieved = the method's bytes per step launch / the launch's HIP-event time; the fused
    # kernel itself moves fewer (it touches the accumulator only on every third step):
    # reported beside it as kernel_bytes_per_launch
    step_ms, kernel_bytes = gs.gs_plan_time_step(plan, reps=10)
    plan.set_kernel(gs.GS_KERNEL_CLENSHAW)   # the same polynomial by Clenshaw's recurrence, same launch shape
    clen_ms, clen_bytes = gs.gs_plan_time_step(plan, reps=10)
    plan.set_kernel(gs.GS_KERNEL_CHEBYSHEV)
    alg_bytes = method_step_bytes(n, g.nnz, P, K)
    achieved = alg_bytes / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic(shape, n, g.nnz, P)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": "cheb_step_kernel (forward form; average launch of a K-step application)", "avg_ms": round(step_ms, 5),
                "algorithmic_bytes_per_launch": int(alg_bytes),
                "algorithmic_bytes_rule": "per step 4(n+1) + 8 nnz + 4n (CSR, degrees) + 20nB (T_{k-1} gathered once, "
                                          "T_{k-2}, T_k, accumulator read + write), 12nB at k = 1; averaged over K",
                "kernel_bytes_per_launch": int(kernel_bytes),
                "kernel_gbs": round(kernel_bytes / (step_ms * 1e-3) / 1e9, 1),
                "clenshaw_form": {"avg_ms": round(clen_ms, 5), "kernel_bytes_per_launch": int(clen_bytes),
                                  "over_accumulating_form": round(clen_ms / step_ms, 4)}}
    log(f"[roofline] step {step_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic ({achieved / PEAK_HBM_GBS:.1%}); "
        f"kernel's own bytes {roofline['kernel_gbs']:.0f} GB/s")

    # plain streaming copy on the same device: achievable bandwidth reference
    nbytes = 2 << 30
    src = torch.empty(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        gs.gs_stream_copy(src, dst)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        gs.gs_stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roofline["frac_of_copy_peak"] = round(achieved / copy_gbs, 4)
    if traffic:
        roofline["traffic_gbs"] = round(traffic / (step_ms * 1e-3) / 1e9, 1)

    # gather reference: the rows the step kernel gathers (one 128-byte row of
    # the n x 32 operand per nonzero, by the graph's own column indices), with
    # nothing else in the kernel; and the same count by uniform random indices
    gather_ref = None
    if P == 32:
        _, col, _, _ = g.export()
        m = len(col)
        idx_sets = {"csr_columns": torch.from_numpy(col.astype(np.int32)).to(dev),
                    "uniform_random": torch.randint(0, n, (m,), dtype=torch.int32,
                                                    generator=torch.Generator().manual_seed(11)).to(dev)}
        Xop = mu.view(n, 32)
        gout = torch.empty((m + 31) // 32 * 32, device=dev)
        gather_ref = {"rows_per_pass": m, "bytes_per_pass": m * 128}
        for name, idx in idx_sets.items():
            for _ in range(2):
                gs.gs_stream_gather(Xop, idx, gout)
            e0.record()
            for _ in range(10):
                gs.gs_stream_gather(Xop, idx, gout)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 10
            gather_ref[name] = {"us": round(us, 1), "gbs": round(m * 128 / (us * 1e-6) / 1e9, 1)}
        gather_ref["step_kernel_us"] = round(step_ms * 1e3, 1)
        gather_ref["step_over_gather"] = round(step_ms * 1e3 / gather_ref["csr_columns"]["us"], 3)
        log(f"[gather] csr columns {gather_ref['csr_columns']['us']:.1f} us "
            f"({gather_ref['csr_columns']['gbs']:.0f} GB/s), random {gather_ref['uniform_random']['us']:.1f} us; "
            f"step {step_ms * 1e3:.1f} us")
        del idx_sets, gout

    # ---------------------------------------------------------------- plain single-RHS form
    plain = None
    if not args.no_plain:
        plan1 = gs.Plan(g, K, 1, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=TUNE_CACHE)
        gs.gs_gather_columns(Hdev, dev_batches[0][0], mu)
        gs.gs_gather_columns(Hdev, dev_batches[0][1], nu)
        mu1 = mu[:, :1].contiguous()
        nu1 = nu[:, :1].contiguous()
        ck1 = torch.empty(gs.ckpt_floats(plan1, J, ce), device=dev)
        g1m = torch.empty(n, device=dev)

        def step1():
            gs.gs_sinkhorn(plan1, lam, t, mu1, nu1, J, ckpt_every=ce, ckpt=ck1)
            gs.gs_sinkhorn_backward(plan1, lam, t, mu1, nu1, J, ce, ck1, [1.0], grad_mu=g1m)

        step1()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        step1()
        torch.cuda.synchronize()
        t1 = time.perf_counter() - w0
        s1_ms, s1_bytes = gs.gs_plan_time_step(plan1, reps=10)
        plain = {"applies_per_s": round(4 * J / t1, 1), "ms_per_pair_fwd_bwd": round(t1 * 1e3, 2),
                 "plan": plan1.describe(), "step_us": round(s1_ms * 1e3, 1),
                 "step_gbs_algorithmic": round(method_step_bytes(n, g.nnz, 1, K) / (s1_ms * 1e-3) / 1e9, 1),
                 "step_gbs_kernel_bytes": round(s1_bytes / (s1_ms * 1e-3) / 1e9, 1)}
        log(f"[plain] B=1 fwd+bwd {t1:.2f}s -> {4 * J / t1:.0f} applies/s")

    extras = None
    if not args.no_extras:
        extras = extra_workloads(gs, synth, np, torch, dev)

    # ---------------------------------------------------------------- oracle on the host
    cpu = None
    if not args.no_cpu_baseline:
        log("[cpu] timing the oracle ...")
        gs.gs_gather_columns(Hdev, dev_batches[0][0], mu)
        gs.gs_gather_columns(Hdev, dev_batches[0][1], nu)
        rp_, col_, w_, _ = g.export()
        cpu = cpu_baseline(rp_, col_, w_, K, t, lam, mu[:, :1].cpu().numpy(), nu[:, :1].cpu().numpy(),
                           inputs["csr_sha256"])
        del rp_, col_, w_
        log(f"[cpu] {cpu['value']:.3f} applies/s")

    other_graphs = None
    if not args.no_other_graphs:
        del ckpt
        other_graphs = roofline_on_other_graphs(gs, synth, np, torch, dev, K, P)
        roofline["same_kernel_other_graphs"] = other_graphs

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "heat-kernel applies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("50 Gaussian clusters x %d on a 2-D spline surface in R^100, sigma 0.1; "
                                "symmetrised k=%d kNN; K=%d, t=%g; J=%d Sinkhorn iterations; "
                                "%d pairs per step from the 256x256 pair matrix, gathered from the resident histograms; forward + reverse sweep (%s); "
                                "pair gradients summed into the total's gradient for each of the 256 histograms"
                                % (args.per_cluster, args.knn, K, t, J, P,
                                   "from recorded denominators" if ce == gs.GS_RECORD_ALL
                                   else f"checkpoints every {ce}, segments recomputed")),
                   "n": n, "nnz": g.nnz, "lambda_hat": round(lam, 6), "pairs_per_step": P, "K": K, "t": t,
                   "iters": J, "ckpt_every": ce,
                   "reverse_sweep": "recorded denominators" if ce == gs.GS_RECORD_ALL else f"checkpoints every {ce}",
                   "plan": shape},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sinkhorn_iters_per_s": round(P * J / (ms_per_step / 1e3), 1),
        "recompute_applies_per_step": 0 if ce == gs.GS_RECORD_ALL else P * 2 * J,
        "checkpointed_form": ckpt_fig,
        "step_kernel_gbs_algorithmic": round(achieved, 1),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "gather_reference": gather_ref,
        "plain_single_rhs": plain,
        "speedup_batched_vs_plain": round(value / plain["applies_per_s"], 2) if plain else None,
        "graph_build_s": round(t_graph, 2),
        "other_workloads": extras,
        "results_finite": bool(finite),
        "inputs": inputs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

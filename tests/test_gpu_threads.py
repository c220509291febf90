"""Two plans used from two host threads at once, each on its own stream.

Each plan owns its workspace and captured graphs; graph capture is
thread-local and the error text is per thread; the graph is shared read-only.
So Algorithm 1 plus the reverse sweep (recorded denominators) run three
times on each thread concurrently give bitwise the results of the same calls
made one after the other, and a failed call on one thread leaves the other
thread's last-error text empty.  Two threads autotuning against one cache
file leave it a valid cache (whole-file replace: the last writer wins).
"""
import json
import threading

import numpy as np
import pytest
import torch

import synth
from gpu_common import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


def _inputs(n, B, seed):
    rng = np.random.default_rng(seed)
    mu = synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.3)
    nu = synth.random_dense_like(n, B, rng, positive=True) * (rng.uniform(size=(n, B)) < 0.3)
    return to_dev(mu / mu.sum(axis=0)), to_dev(nu / nu.sum(axis=0))


def _run(gs, plan, lam, mu, nu):
    n, B = plan.n, plan.B
    K, t, J = plan.K, 1.0, 5
    ckpt = torch.empty(gs.ckpt_floats(plan, J, gs.GS_RECORD_ALL), device="cuda")
    out = gs.gs_sinkhorn(plan, lam, t, mu, nu, J, ckpt_every=gs.GS_RECORD_ALL, ckpt=ckpt, want_floors=True)
    gmu = torch.empty(n * B, device="cuda")
    gt = gs.gs_sinkhorn_backward(plan, lam, t, mu, nu, J, gs.GS_RECORD_ALL, ckpt, np.ones(B), grad_mu=gmu)
    return out["dist"].copy(), out["n_floored"], gmu.cpu().numpy(), gt.copy()


def test_two_plans_on_two_threads(gs):
    n, K = 3000, 16
    arrs = synth.random_local_graph(n, 6, 200, np.random.default_rng(61), hubs=2, hub_degree=900)
    g = gs.gs_graph_from_csr(n, *arrs)
    lam = g.edge_bound
    cases = {"a": (3, _inputs(n, 3, 62)), "b": (8, _inputs(n, 8, 63))}
    ref = {}
    for name, (B, (mu, nu)) in cases.items():
        ref[name] = _run(gs, gs.Plan(g, K, B), lam, mu, nu)
    torch.cuda.synchronize()

    from paper_2211_00805_amd import _lib
    results, errors, failures = {}, {}, []
    barrier = threading.Barrier(len(cases), timeout=120)

    def worker(name):
        try:
            B, (mu, nu) = cases[name]
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                plan = gs.Plan(g, K, B)
                barrier.wait()
                results[name] = [_run(gs, plan, lam, mu, nu) for _ in range(3)]
                if name == "a":
                    try:
                        gs.gs_sinkhorn(plan, -1.0, 1.0, mu, nu, 2)
                        failures.append("negative lambda_hat accepted")
                    except gs.GeoSinkError:
                        pass
                barrier.wait()   # thread a has failed a call: b's own error text must still be empty
                errors[name] = _lib.lib.gs_last_error().decode()
            stream.synchronize()
        except Exception as e:  # reported by the main thread
            failures.append(f"{name}: {e!r}")

    threads = [threading.Thread(target=worker, args=(name,)) for name in cases]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert not failures, failures
    assert errors["a"] != "" and errors["b"] == ""
    for name in cases:
        for run in results[name]:
            for got, want in zip(run, ref[name]):
                assert np.array_equal(np.asarray(got), np.asarray(want)), name


def test_concurrent_autotuning_leaves_a_valid_cache(gs, tmp_path):
    n = 3000
    arrs = synth.random_local_graph(n, 6, 200, np.random.default_rng(64))
    g = gs.gs_graph_from_csr(n, *arrs)
    cache = str(tmp_path / "tune.json")
    plans = {}

    def worker(B):
        with torch.cuda.stream(torch.cuda.Stream()):
            plans[B] = gs.Plan(g, 12, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=cache)
        torch.cuda.synchronize()

    threads = [threading.Thread(target=worker, args=(B,)) for B in (4, 16)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    with open(cache) as f:
        entries = json.load(f)
    assert 1 <= len(entries) <= 2
    for key, val in entries.items():
        assert key.endswith(":B=4") or key.endswith(":B=16")
        assert len(val.split(",")) == 5   # vec, S, C, XCD order, CSR hint
    assert not [p for p in tmp_path.iterdir() if ".tmp." in p.name]
    for key in entries:
        B = int(key.split("B=")[1])
        again = gs.Plan(g, 12, B, flags=gs.GS_PLAN_AUTOTUNE, tune_cache=cache)
        assert "origin=cache" in again.describe()
        assert again.describe().split(" origin")[0] == plans[B].describe().split(" origin")[0]

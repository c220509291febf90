"""Host checks of the stored full-size oracle values (tests/golden/fullsize_*).

The values were written by tests/golden/make_fullsize.py, which calls only the
oracle and the seeded generators.  Here, without a GPU and without re-running
the float64 oracle at full size: the histograms and the 1M graph the GPU tests
rebuild have the stored digests; every stored array has the length of its
support; the float64 reference gradient agrees with the oracle's own central
differences to 1e-6 (relative) on the 16 sampled coordinates and in t; the
stored lambda_hat brackets the spectrum by the oracle's definition
(lambda_max <= lambda_hat = 1.01 lambda_max <= edge bound); the oracle's own
runs converge (small marginal violation) and floor nothing.
"""
import json
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, f"fullsize_{name}.json")) as f:
        rec = json.load(f)
    return rec, dict(np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz")))


def graph_ok(g):
    assert g["lambda_max"] > 0
    assert g["lambda_hat"] == pytest.approx(1.01 * g["lambda_max"], rel=1e-15)
    assert g["lambda_max"] <= g["lambda_hat"] <= g["edge_bound"]


def test_curve_fixture():
    rec, arr = load("curve")
    graph_ok(rec["graph"])
    assert rec["graph"]["n_components"] == 1
    mu = synth.curve_pair_workload(per_cluster=5000)[2]
    assert synth.sha256(mu) == rec["mu_sha256"]
    assert [r["t"] for r in rec["runs"]] == [0.5, 2.0, 8.0]
    for r in rec["runs"]:
        row = arr[f"row_t{r['t']}"]
        assert row.shape == ((mu > 0).sum(),)
        assert r["n_floored"] == 0 and r["marg_row"] < 1e-6
        # the row marginal is the plan's: its mass equals mu's up to the violation
        assert abs(row.astype(np.float64).sum() - mu.astype(np.float64).sum()) <= r["marg_row"] + 1e-6


def test_barycenter_fixture():
    rec, arr = load("bary")
    graph_ok(rec["graph"])
    graph_ok(rec["twin_graph"])
    assert arr["p_full"].shape == (rec["graph"]["n"],) and arr["p_twin"].shape == (rec["twin_graph"]["n"],)
    assert rec["full"]["J"] == 20 and rec["twin"]["J"] == 300
    assert rec["full"]["n_floored"] == 0 and rec["twin"]["n_floored"] == 0
    assert np.all(arr["p_full"] > 0) and np.all(arr["p_twin"] > 0)
    assert abs(rec["twin"]["mass"] - 1.0) < 1e-3   # converged IBP keeps unit mass


def test_gradient_fixture_against_central_differences():
    """The float64 reverse-mode gradient against the oracle's own central differences.

    A central difference with step h carries the rounding error of D divided
    by h: D (about 60-110 here) comes out of J = 200 float64 iterations
    accurate to a few tens of ulp, so at the workload's relative step 1e-4 on
    small weights (h down to 6e-10) that term reaches 1e-5 relative.  Checked,
    at both relative steps (1e-4, the workload's, and 1e-3, where that term is
    ten times smaller and truncation stays near 1e-8): every coordinate within
    1e-6 relative plus 128 ulp of D over 2h; at the step 1e-3, every
    coordinate whose rounding term is below 1e-6 relative within 1e-6
    relative outright; the agreement improves with the larger step (the
    differences' rounding, not the reference, sets it); d/dt within 1e-6.
    """
    rec, arr = load("grad")
    graph_ok(rec["graph"])
    assert rec["ref_vs_fd_max_rel"]["t"] <= 1e-6
    assert len(rec["fd_mu"]) == 16 and {r["pair"] for r in rec["fd_mu"]} == {0, 1, 2, 3}
    eps = np.finfo(np.float64).eps
    pinned, err4, err3 = 0, [], []
    for r in rec["fd_mu"]:
        D = rec[f"ref_{r['pair']}"]["D"]
        assert abs(r["ref"] - r["fd"]) <= 1e-6 * abs(r["fd"]) + 128 * eps * abs(D) / (2 * r["h"]), r
        err4.append(abs(r["ref"] - r["fd"]) / abs(r["fd"]))
        fd3, h3 = r["fd_rel1e-3"], r["h_rel1e-3"]
        rounding3 = 128 * eps * abs(D) / (2 * h3)
        assert abs(r["ref"] - fd3) <= 1e-6 * abs(fd3) + rounding3, r
        err3.append(abs(r["ref"] - fd3) / abs(fd3))
        if rounding3 < 1e-6 * abs(fd3):
            assert abs(r["ref"] - fd3) <= 1e-6 * abs(fd3), r
            pinned += 1
    assert pinned >= 12
    assert np.median(err3) < np.median(err4) / 3
    for c in rec["ref_pairs"]:
        ref = rec[f"ref_{c}"]
        assert ref["D"] == pytest.approx(ref["D_grad_run"], rel=1e-12)
        assert ref["n_floored"] == 0
        assert arr[f"dmu_{c}"].shape == arr[f"row_{c}"].shape


def test_local1m_fixture_and_inputs():
    rec, arr = load("local1m")
    g = rec["graph"]
    graph_ok(g)
    rp, col, w = synth.local_graph_1m()
    assert synth.sha256(rp) == g["rowptr_sha256"] and synth.sha256(col) == g["col_sha256"]
    assert synth.sha256(w) == g["w_sha256"]
    mu, nu = synth.loguniform_pair_batch(rp.shape[0] - 1, 32, 5000, 200000, 10)
    assert synth.sha256(mu) == rec["mu_sha256"] and synth.sha256(nu) == rec["nu_sha256"]
    for c in rec["ref_pairs"]:
        ref = rec[f"ref_{c}"]
        assert arr[f"dmu_{c}"].shape == ((mu[:, c] > 0).sum(),)
        assert arr[f"dnu_{c}"].shape == ((nu[:, c] > 0).sum(),)
        assert ref["D"] == pytest.approx(ref["D_grad_run"], rel=1e-12)
        assert ref["n_floored"] == 0

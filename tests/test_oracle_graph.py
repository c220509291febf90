"""Pins for the oracle's kNN affinity graph, Laplacian and spectral bounds."""
import json
import os

import numpy as np
import pytest
from scipy.linalg import eigvalsh
from scipy.spatial import cKDTree

import synth
from oracle import graph, spectrum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_knn_lists_match_kdtree():
    X = np.random.default_rng(0).standard_normal((600, 5))
    idx, d2 = graph.knn_lists(X, 7, block=128)
    dd, ii = cKDTree(X).query(X, k=8)
    np.testing.assert_array_equal(idx, ii[:, 1:])
    np.testing.assert_allclose(d2, dd[:, 1:] ** 2, rtol=1e-12)


def test_knn_ties_go_to_lower_index():
    X = np.arange(10, dtype=np.float64)[:, None]       # integer points on a line
    idx, _ = graph.knn_lists(X, 3)
    assert list(idx[5]) == [4, 6, 3]                   # 3 and 7 tie at distance 2
    assert list(idx[0]) == [1, 2, 3]


def test_hand_worked_line_graph():
    with open(os.path.join(GOLDEN, "knn_line.json")) as f:
        g = json.load(f)
    A, info = graph.knn_graph(np.array(g["points"], dtype=np.float64)[:, None], g["k"])
    assert info["median"] == pytest.approx(g["median"], rel=1e-15)
    dense = A.toarray()
    np.testing.assert_allclose(dense, np.array(g["adjacency"]), rtol=1e-15, atol=0)


def test_graph_structure_properties():
    X, labels = synth.clusters_on_curve(6, 150, dim=8, sigma=0.1, n_knots=5, workload=7)
    A, info = graph.knn_graph(X, 10)
    n = X.shape[0]
    assert (A != A.T).nnz == 0
    assert A.diagonal().max() == 0
    deg_out = np.diff(A.indptr)
    assert deg_out.min() >= 10
    # every directed kNN edge is present, and nothing else
    rows = np.repeat(np.arange(n), 10)
    assert np.all(A[rows, info["knn_idx"].ravel()] > 0)
    union = set(zip(rows.tolist(), info["knn_idx"].ravel().tolist()))
    union |= {(j, i) for i, j in union}
    coo = A.tocoo()
    assert set(zip(coo.row.tolist(), coo.col.tolist())) == union
    # exp(-d^2/m^2) >= e^{-1} exactly when d <= m: half of the directed distances
    d = info["directed_dist"]
    assert np.sum(d < info["median"]) == d.size // 2
    w = np.asarray(A[rows, info["knn_idx"].ravel()]).ravel()
    assert np.sum(w > np.exp(-1.0)) == d.size // 2
    assert info["n_components"] == 1


def test_two_far_clusters_are_two_components():
    rng = np.random.default_rng(1)
    X = np.concatenate([rng.standard_normal((50, 3)), 100.0 + rng.standard_normal((50, 3))])
    _, info = graph.knn_graph(X, 5)
    assert info["n_components"] == 2


def test_laplacian_rows_sum_to_zero():
    X = np.random.default_rng(2).standard_normal((200, 3))
    A, _ = graph.knn_graph(X, 6)
    L = graph.laplacian(A)
    assert np.abs(np.asarray(L.sum(axis=1))).max() < 1e-13


def test_lambda_max_and_bounds():
    X = np.random.default_rng(3).standard_normal((400, 4))
    A, _ = graph.knn_graph(X, 8)
    L = graph.laplacian(A)
    lm = spectrum.lambda_max(L)
    assert lm == pytest.approx(eigvalsh(L.toarray())[-1], rel=1e-12)
    # the ARPACK path agrees with the dense one
    assert spectrum.lambda_max(L, dense_limit=10) == pytest.approx(lm, rel=1e-9)
    eb = spectrum.edge_bound(A)
    assert lm <= eb <= spectrum.gershgorin_bound(A) + 1e-12


def test_complete_graph_spectrum():
    n = 25
    A = graph.csr_from_arrays(n, *synth.complete_graph(n))
    L = graph.laplacian(A)
    assert spectrum.lambda_max(L) == pytest.approx(n, rel=1e-13)
    assert spectrum.edge_bound(A) == pytest.approx(2 * (n - 1))


def test_knn_row_ranges_assemble_the_full_search():
    """knn_lists over row ranges, concatenated, equals the single search; knn_graph
    built from those lists equals the graph built directly (weights by
    gaussian_weights of the union's pairs)."""
    X = np.random.default_rng(3).standard_normal((700, 6))
    full, d2 = graph.knn_lists(X, 9)
    parts = [graph.knn_lists(X, 9, block=128, rows=(lo, min(700, lo + 256)))[0] for lo in range(0, 700, 256)]
    assert np.array_equal(np.concatenate(parts), full)
    A, info = graph.knn_graph(X, 9)
    A2, _ = graph.knn_graph(X, 9, knn_idx=np.concatenate(parts))
    assert (A != A2).nnz == 0
    coo = A.tocoo()
    w = graph.gaussian_weights(X, coo.row, coo.col, info["median"])
    assert np.array_equal(w, coo.data)
    with pytest.raises(ValueError):
        graph.knn_lists(X, 9, rows=(600, 800))

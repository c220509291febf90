"""Host-side checks of the library's nearest-neighbour scores and pair batching.

The scores (average-rank Spearman, Pearson, precision at k) are compared with
the oracle's, which uses scipy's statistics, on random matrices with ties;
no GPU call is made.
"""
import numpy as np
import pytest

from oracle import pairwise as opw


@pytest.fixture(scope="module")
def pw():
    from paper_2211_00805_amd import pairwise
    return pairwise


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_scores_match_scipy_definitions(pw, seed):
    rng = np.random.default_rng(seed)
    m = 12
    pts = rng.standard_normal((m, 2))
    truth = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    D = truth ** 2 + rng.uniform(0, 0.5, (m, m))
    D = np.round(0.5 * (D + D.T), 1)          # ties
    np.fill_diagonal(D, 0)
    a, b = pw.nn_scores(D, truth), opw.nn_scores(D, truth)
    assert a["spearman"] == pytest.approx(b["spearman"], abs=1e-12)
    assert a["pearson"] == pytest.approx(b["pearson"], abs=1e-12)
    assert a["p_at_5"] == b["p_at_5"]


def test_pair_list():
    p = __import__("paper_2211_00805_amd").pair_list(4)
    assert p.tolist() == [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]
    assert len(__import__("paper_2211_00805_amd").pair_list(15, diagonal=True)) == 120

"""The measurement helpers compute what they state: gs_stream_copy copies
exactly, gs_stream_gather sums each run of 32 gathered rows (entries outside
[0, n) read row 0), for a ragged last run."""
import numpy as np
import pytest
import torch

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2211_00805_amd as g
    return g


def test_stream_copy_is_exact(gs):
    src = torch.randn(1_000_003, device="cuda")
    dst = torch.empty_like(src)
    gs.gs_stream_copy(src, dst)
    assert torch.equal(src, dst)


def test_stream_gather_sums_runs_of_rows(gs):
    n, m = 1000, 100
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (n, 32)).astype(np.float32)
    idx = rng.integers(0, n, m).astype(np.int32)
    idx[[5, 70]] = [-4, n + 9]           # out of range: row 0
    Xd = torch.from_numpy(X).cuda()
    out = torch.empty((m + 31) // 32 * 32, device="cuda")
    gs.gs_stream_gather(Xd, torch.from_numpy(idx).cuda(), out)
    got = out.cpu().numpy().reshape(-1, 32)
    eff = np.where((idx >= 0) & (idx < n), idx, 0)
    for r in range(got.shape[0]):
        ref = X[eff[32 * r:32 * (r + 1)]].astype(np.float64).sum(axis=0)
        np.testing.assert_allclose(got[r], ref, rtol=1e-5, atol=1e-5)

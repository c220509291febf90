"""Shared helpers for the GPU parity tests (graphs as CSR arrays, tolerances)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import graph as ograph
from oracle import spectrum

U32 = 2.0 ** -24  # unit roundoff of float32


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def oracle_csr(X, k):
    """Oracle kNN graph, its float32 CSR arrays and the float64 Laplacian of those float32 weights."""
    A, info = ograph.knn_graph(X, k)
    rp = A.indptr.astype(np.int32)
    col = A.indices.astype(np.int32)
    w32 = A.data.astype(np.float32)
    A32 = ograph.csr_from_arrays(A.shape[0], rp, col, w32.astype(np.float64))
    return (rp, col, w32), ograph.laplacian(A32), info, A


def csr_laplacian(n, arrs):
    return ograph.laplacian(ograph.csr_from_arrays(n, *[np.asarray(a) for a in arrs]))


def lam_hat_of(L, safety=1.01):
    return safety * spectrum.lambda_max(L)


def heat_tol(K, xmax):
    """Max-abs tolerance of a float32 degree-K application against float64.

    Each of the K steps rounds O(1) float32 operations on values bounded by
    max|X| (|T_k(y)| <= 1 on the spectrum); the bound 8 K u max|X| leaves a
    factor of a few over the observed error.
    """
    return 8.0 * K * U32 * xmax + 1e-30


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)

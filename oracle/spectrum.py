"""Largest Laplacian eigenvalue and its classical upper bounds (oracle, float64).

The Chebyshev expansion in Sec. "Chebyshev Polynomials" assumes the spectrum
of the operator it expands lies in [0, 2]; the paper is silent on how the
largest eigenvalue is found.  Reading: the operator is rescaled by an explicit
scalar lam_hat >= lambda_max(L); this module gives lambda_max exactly (dense
or ARPACK) and the edge bound max_{(i,j) in E} (d_i + d_j), which is always
>= lambda_max for non-negative weights.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import eigvalsh
from scipy.sparse.linalg import eigsh


def lambda_max(L: sp.spmatrix, dense_limit: int = 3000) -> float:
    """Largest eigenvalue of the symmetric PSD Laplacian."""
    n = L.shape[0]
    if n <= dense_limit:
        return float(eigvalsh(L.toarray())[-1])
    val = eigsh(sp.csr_matrix(L, dtype=np.float64), k=1, which="LA", tol=1e-10,
                return_eigenvectors=False)
    return float(val[0])


def edge_bound(A: sp.spmatrix) -> float:
    """max over edges (i, j) of d_i + d_j (an upper bound on lambda_max(D - A))."""
    A = sp.coo_matrix(A)
    deg = np.asarray(sp.csr_matrix(A).sum(axis=1)).ravel()
    if A.nnz == 0:
        return 0.0
    return float(np.max(deg[A.row] + deg[A.col]))


def gershgorin_bound(A: sp.spmatrix) -> float:
    """2 * max degree (a looser upper bound on lambda_max(D - A))."""
    deg = np.asarray(sp.csr_matrix(A).sum(axis=1)).ravel()
    return float(2.0 * deg.max())

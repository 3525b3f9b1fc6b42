"""Brute-force symbolic Cholesky: TEST INFRASTRUCTURE ONLY.

Boolean Gaussian elimination on the pattern of a symmetric matrix: after
eliminating column j, every pair of rows below j that are both nonzero in
column j becomes nonzero. The resulting lower pattern is the structure of
the Cholesky factor L under the given ordering (no cancellation assumed).
It is O(n^3) on dense boolean arrays and meant for n up to a few thousand.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def k_pattern(pat) -> sp.csr_matrix:
    """Boolean pattern of K = W + diag + J^T J (full symmetric)."""
    n = pat.n
    Wl = sp.csr_matrix((np.ones(pat.nnz_w), pat.w_colind, pat.w_rowptr), shape=(n, n))
    J = sp.csr_matrix((np.ones(pat.nnz_j), pat.j_colind, pat.j_rowptr), shape=(pat.m, n))
    K = (Wl + Wl.T + sp.eye(n) + J.T @ J).tocsr()
    K.data[:] = 1.0
    return K


def cholesky_structure(Kpat, perm=None) -> np.ndarray:
    """Dense boolean lower-triangular structure of L (diagonal included)."""
    A = (Kpat.toarray() != 0)
    if perm is not None:
        A = A[np.ix_(perm, perm)]
    n = A.shape[0]
    A = A | np.eye(n, dtype=bool)
    for j in range(n):
        rows = np.nonzero(A[j + 1:, j])[0] + j + 1
        if len(rows):
            A[np.ix_(rows, rows)] = True
    return np.tril(A)


def stats(Lstruct: np.ndarray) -> dict:
    """nnz(L) with diagonal, sum over columns of (column count)^2, and the etree."""
    counts = Lstruct.sum(axis=0)
    n = Lstruct.shape[0]
    parent = np.full(n, -1)
    for j in range(n):
        below = np.nonzero(Lstruct[j + 1:, j])[0]
        if len(below):
            parent[j] = below[0] + j + 1
    return dict(nnz_l=int(counts.sum()), sum_c2=int((counts.astype(np.int64) ** 2).sum()),
                counts=counts, parent=parent)

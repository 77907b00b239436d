"""Memory usage of the factors, Eq. 15 of the paper's experimental settings:
(nnz(C) + nnz(U) + nnz(R)) / nnz(X).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Reading: nnz(U) is counted structurally.  Kept fibers that share a row are
linked; R^T R is block diagonal over the connected groups (after a
permutation), so is its inverse U, and a group of g fibers has a dense g x g
inverse block, contributing g^2.  (Counting |U_ab| > 0 of a computed inverse
would depend on rounding where the exact entry is zero.)
"""
from __future__ import annotations

import numpy as np


def structural_nnz_U(R) -> int:
    """Sum of g^2 over the groups of columns of R linked by shared rows."""
    R = np.asarray(R)
    k = R.shape[1]
    parent = list(range(k))

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for r in range(R.shape[0]):
        cols = np.flatnonzero(R[r] != 0.0)
        for a, b in zip(cols[:-1], cols[1:]):
            x, y = root(int(a)), root(int(b))
            if x != y:
                parent[max(x, y)] = min(x, y)
    sizes = np.bincount([root(a) for a in range(k)], minlength=k) if k else np.zeros(0, int)
    return int((sizes.astype(np.int64) ** 2).sum())


def memory_usage(R, C, nnz_X):
    """(nnz(C), nnz(U), nnz(R), usage) with C = R^T X_(alpha) (dense or sparse)."""
    nnz_R = int(np.count_nonzero(np.asarray(R)))
    nnz_C = int(C.count_nonzero()) if hasattr(C, "count_nonzero") else int(np.count_nonzero(C))
    nnz_U = structural_nnz_U(R)
    return nnz_C, nnz_U, nnz_R, (nnz_C + nnz_U + nnz_R) / nnz_X


def sparse_core(R, u):
    """C_(alpha) = R^T X_(alpha) (the last step of Algorithm 1) as a sparse
    matrix over the non-empty fibers of the unfolding `u` (u.mat, columns in
    ascending fiber id): compressed-column (indptr, indices, data) with row
    indices ascending in each column and entries whose value is exactly zero
    dropped.  The product is scipy's sparse matrix product."""
    import scipy.sparse as sp
    C = (sp.csr_matrix(np.asarray(R)).T @ u.mat).tocsc()
    C.eliminate_zeros()
    C.sort_indices()
    return C.indptr.astype(np.int64), C.indices.astype(np.int32), C.data.astype(np.float64)

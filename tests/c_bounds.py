"""Entrywise error bound of the library's CTD-D C against its closed form
(shared by the GPU tests; not a test module)."""
import numpy as np

from oracle import ctd as ora


def core_error_bound(inputs, ncols_after, rank_after, cols, R, Q, M, ref, batch, u):
    """Bound on |C - C_ref| for the columns `cols` of C, from how the library forms C
    (a running error bound of its arithmetic; u is the unit roundoff of C's element
    type: 2^-53 for a float64 C, 2^-24 for a float32 C).

    inputs: the initial tensor and the slices, in order; ncols_after[t + 1] and
    rank_after[t + 1]: the columns of C and the kept fibers after slice t (index 0:
    after the initial CTD-S); batch: slices per update call.

    An entry (a, c) whose row a was held when column c arrived is r_a^T x_c: bound
    (nnz_c + 4) u |r_a|^T |x_c|.  A later row is a cross term of Eq. 13: with K the
    rank of the pass that formed it (the rank at the start of the batch for columns
    held before the batch, the rank after the column's slice for columns of the same
    batch), the library forms y = M_K (Q_K^T r_a) and the sum y^T C[:K, c], so the
    entry carries (K + 8) u sum_j |y_j| |C_jc| of its own rounding (the products, the
    sum and y's rounding to C's type) plus sum_j |y_j| B_jc of the errors already in
    C[:K, c].  Every entry adds u |C_ac| for its storage."""
    cols = np.asarray(cols)
    ncols_after = np.asarray(ncols_after)
    rank_after = np.asarray(rank_after)
    k = R.shape[1]
    tau = np.searchsorted(ncols_after, cols, side="right") - 1     # -1: initial tensor
    row_step = np.searchsorted(rank_after, np.arange(k), side="right") - 1
    X = np.zeros((R.shape[0], len(cols)))
    unf = {}
    for j, (c, t) in enumerate(zip(cols.tolist(), tau.tolist())):
        if t not in unf:
            T = inputs[t + 1]
            unf[t] = ora.unfold(T.dims, T.idx, T.val, 0)
        X[:, j] = unf[t].column(int(c - (ncols_after[t] if t >= 0 else 0)))
    nnz_c = np.count_nonzero(X, axis=0)
    W = Q.T @ R                                                    # w_a = Q^T r_a
    absC = np.abs(ref)
    B = (np.abs(R).T @ np.abs(X)) * (nnz_c + 4) * u                # direct entries
    for a in range(k):
        ta = row_step[a]
        held = ta <= tau
        if np.all(held):
            continue
        bs = ta - ta % batch
        Ks = np.where(tau < bs, rank_after[bs], rank_after[tau + 1])
        for K in np.unique(Ks[~held]).tolist():
            sel = (~held) & (Ks == K)
            y = np.abs(M[:K, :K] @ W[:K, a])
            B[a, sel] = (K + 8) * u * (y @ absC[:K][:, sel]) + y @ B[:K][:, sel]
    return B + u * absC

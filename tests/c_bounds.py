"""Entrywise error bound of the library's CTD-D C against its closed form
(shared by the GPU tests; not a test module)."""
import numpy as np

from oracle import ctd as ora


def core_error_bound(inputs, ncols_after, rank_after, cols, R, Q, M, ref, batch, u):
    """Bound on |C - C_ref| for the columns `cols` of C, from how the library forms C
    (a first-order running error bound of its arithmetic; u is the unit roundoff of
    C's element type: 2^-53 for a float64 C, 2^-24 for a float32 C).

    inputs: the initial tensor and the slices, in order; ncols_after[t + 1] and
    rank_after[t + 1]: the columns of C and the kept fibers after slice t (index 0:
    after the initial CTD-S); batch: slices per update call; R, Q, M: the library's
    kept fibers, orthonormal basis and upper-triangular M (Q = R M).

    An entry (a, c) whose row a was held when column c arrived is r_a^T x_c: bound
    (nnz_c + 4) u |r_a|^T |x_c|.  A later row is a cross term of Eq. 13, formed by
    the pass of rank K (the rank at the start of the batch for columns held before
    the batch, the rank after the column's slice for columns of the same batch) as
    y^T C[:K, c] with y = M_K w and w = Q_K^T r_a the filter's coefficients.  In
    exact arithmetic that is (R_K M_K w)^T P x_c = r_a^T P x_c, so the entry carries
      (K + 8) u sum_j z_j |C_jc|     its rounding: the products and the sum, y
                                     (|y - M_K w| <= gamma_K |M_K| |w|) and w
                                     (about u |Q_K|^T |r_a|), z = |M_K| |Q_K|^T |r_a|;
      (F_K |w|)^T |P_K x_c|          the inexact relation Q_K = R_K M_K of the
                                     computed factors, F = |Q - R M| + k u |R| |M|;
      sum_j |y_j| B_jc               the errors already in C[:K, c].
    Every entry adds u |C_ac| for its storage."""
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
    PX = np.zeros_like(X)                                          # |P_tau x_c|
    for t in np.unique(tau).tolist():
        sel = tau == t
        Kt = rank_after[t + 1]
        PX[:, sel] = np.abs(Q[:, :Kt] @ (Q[:, :Kt].T @ X[:, sel]))
    W = Q.T @ R                                                    # w_a = Q^T r_a
    Wabs = np.abs(Q).T @ np.abs(R)
    absM = np.abs(M)
    F = np.abs(Q - R @ M) + k * u * (np.abs(R) @ absM)
    absC = np.abs(ref)
    B = (np.abs(R).T @ np.abs(X)) * (nnz_c + 4) * u                # direct entries
    for ta in np.unique(row_step).tolist():
        if ta < 0:
            continue
        rows = np.nonzero(row_step == ta)[0]
        held = ta <= tau
        bs = ta - ta % batch
        Ks = np.where(tau < bs, rank_after[bs], rank_after[tau + 1])
        for K in np.unique(Ks[~held]).tolist():
            csel = np.nonzero((~held) & (Ks == K))[0]
            Y = np.abs(M[:K, :K] @ W[:K][:, rows])                 # K x rows
            Z = absM[:K, :K] @ Wabs[:K][:, rows]
            rel = (F[:, :K] @ np.abs(W[:K][:, rows])).T @ PX[:, csel]
            for i, a in enumerate(rows.tolist()):
                B[a, csel] = ((K + 8) * u * (Z[:, i] @ absC[:K][:, csel]) + rel[i]
                              + Y[:, i] @ B[:K][:, csel])
    return B + u * absC

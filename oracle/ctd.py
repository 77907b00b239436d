"""Plain float64 CPU oracle for CTD (Compact Tensor Decomposition).

TEST INFRASTRUCTURE ONLY.  Only tests/, the package smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code,
table or helper with the HIP library; the two meet only in the seeded input
generators of `workloads/`, which hold none of the method's arithmetic.

What is computed, by section of the paper:
  * Section 2.1: mode-alpha fibers, the matricization X_(alpha), the
    Frobenius norm (Eq. 1) and the n-mode product property (Eq. 3).
  * Section 3.1, Algorithm 1 (CTD-S): column distribution, sampling with
    replacement, unique selection, the incremental independence loop that
    grows R and U, and C = X x_alpha R^T.
  * Lemma 2 (Eqs. 4-7): with R0 the sampled fibers, the CTD-S error equals
    the least-squares error min_L ||X_(alpha) - R0 L||_F.
  * Section 3.2, Algorithm 2 (CTD-D): per-slice sampling, extension of R and
    U from the previous step, and the block update of C (Eqs. 8-13) with the
    left-to-right parenthesization of the cross term.
  * Section 4.1, Eq. 14: relative error ||X~ - X||_F^2 / ||X||_F^2.

Readings taken where the paper leaves a choice open (each is also listed in
the design notes of the repository):
  * Column order of X_(alpha): column-major over the remaining modes in
    increasing mode order (mode 1 of a 3-way tensor: column j + k*J), so new
    time slices append trailing columns, as Eqs. 10-11 require.
  * Unique selection (Algorithm 1) lists fibers by ascending column
    index; the independence loop visits them in that order.
  * Sampling with P(i) (Algorithm 1) uses integer-quantized
    weights so that a CPU and a GPU draw identical indices: with
    E = exponent of the largest squared value (largest v^2 < 2^E),
    L = ceil(log2 nnz) and sigma = 62 - L - E, every nonzero contributes
    q = floor(v^2 * 2^sigma) and a fiber's weight is the exact integer sum of
    its q; the total W stays below 2^62.  Draw j takes a 128-bit Philox
    output r and the target t = floor(r * W / 2^128); the drawn column is the
    first one whose inclusive cumulative weight exceeds t.
  * Duplicate draws are merged into one column; the merged column would
    carry the scale sqrt(k / (s p)) of the sampling-with-replacement
    estimators the paper builds on (Section 2.2), with k the multiplicity
    and p the quantized probability.  R itself stays unscaled (actual
    fibers); the scale is reported beside it and changes neither U, C nor
    the error, because the projection onto span(R) ignores column scaling.
  * The independence test (Algorithm 1) skips a fiber when
    ||res|| <= eps ||x||, equality included; the first unique fiber is
    always kept (R starts from it).
  * A tensor with ||X||_F = 0 has no column distribution and is rejected, as
    are duplicate coordinates, out-of-range indices and non-finite values.
"""
from __future__ import annotations

import bisect
import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from .philox import draw_u128


# ---------------------------------------------------------------------------
# Section 2.1: fibers and the mode-alpha matricization
# ---------------------------------------------------------------------------

def fiber_ids(dims, idx, mode) -> np.ndarray:
    """Column index of each nonzero in X_(mode): column-major over the other modes."""
    f = np.zeros(idx.shape[1], dtype=np.int64)
    stride = 1
    for m in range(len(dims)):
        if m == mode:
            continue
        f += idx[m].astype(np.int64) * stride
        stride *= int(dims[m])
    return f


@dataclasses.dataclass
class Unfolding:
    """X_(alpha) restricted to its non-empty columns."""
    n_rows: int            # I_alpha
    n_cols_total: int      # N_alpha
    fids: np.ndarray       # int64 [n_f], ascending column indices of the non-empty fibers
    mat: sp.csc_matrix     # I_alpha x n_f, column j is fiber fids[j], rows ascending
    norm2: float           # ||X||_F^2 (Eq. 1), exactly rounded sum

    @property
    def n_f(self):
        return self.fids.shape[0]

    def column(self, j) -> np.ndarray:
        x = np.zeros(self.n_rows)
        a, b = self.mat.indptr[j], self.mat.indptr[j + 1]
        x[self.mat.indices[a:b]] = self.mat.data[a:b]
        return x


def unfold(dims, idx, val, mode) -> Unfolding:
    """Validate a COO tensor and return its mode-`mode` matricization."""
    dims = tuple(int(d) for d in dims)
    idx = np.asarray(idx)
    val = np.asarray(val, dtype=np.float64)
    if not 0 <= mode < len(dims):
        raise ValueError("mode out of range")
    for m, d in enumerate(dims):
        if idx.shape[1] and (idx[m].min() < 0 or idx[m].max() >= d):
            raise ValueError("index out of range")
    if not np.all(np.isfinite(val)):
        raise ValueError("non-finite value")
    f = fiber_ids(dims, idx, mode)
    r = idx[mode].astype(np.int64)
    order = np.lexsort((r, f))
    f, r, v = f[order], r[order], val[order]
    if f.shape[0] > 1:
        same = (f[1:] == f[:-1]) & (r[1:] == r[:-1])
        if np.any(same):
            raise ValueError("duplicate coordinate")
    fids, start, counts = np.unique(f, return_index=True, return_counts=True)
    indptr = np.zeros(fids.shape[0] + 1, dtype=np.int64)
    indptr[1:] = np.cumsum(counts)
    mat = sp.csc_matrix((v, r, indptr), shape=(dims[mode], fids.shape[0]))
    n_total = 1
    for m, d in enumerate(dims):
        if m != mode:
            n_total *= d
    return Unfolding(dims[mode], n_total, fids, mat, math.fsum((v * v).tolist()))


# ---------------------------------------------------------------------------
# Algorithm 1: column distribution, sampling, unique selection
# ---------------------------------------------------------------------------

def quantized_weights(u: Unfolding):
    """Integer column weights proportional to squared fiber norms.

    Returns (w, W): w[j] is the exact integer weight of fiber j (uint64
    array), W the exact total as a Python int.
    """
    v = u.mat.data
    nnz = v.shape[0]
    v2 = v * v
    vmax2 = float(v2.max())
    if vmax2 == 0.0:
        raise ValueError("tensor has zero Frobenius norm")
    e_max = math.frexp(vmax2)[1]            # vmax2 < 2**e_max
    l_bits = (nnz - 1).bit_length()         # ceil(log2(nnz))
    sigma = 62 - l_bits - e_max
    q = np.array([int(math.ldexp(x, sigma)) for x in v2.tolist()], dtype=np.uint64)
    w = np.add.reduceat(q, u.mat.indptr[:-1]) if nnz else np.zeros(0, np.uint64)
    counts = np.diff(u.mat.indptr)
    w = np.where(counts > 0, w, 0).astype(np.uint64)
    W = int(sum(int(x) for x in w.tolist()))
    assert W < (1 << 62)
    return w, W


def sample_columns(w, W, s, seed, step=0, tensor=0):
    """Positions (into the non-empty fiber list) of s draws, in draw order."""
    cdf = []
    acc = 0
    for x in w.tolist():
        acc += int(x)
        cdf.append(acc)
    out = np.empty(s, dtype=np.int64)
    for j in range(s):
        r = draw_u128(seed, j, step, tensor)
        t = (r * W) >> 128
        out[j] = bisect.bisect_right(cdf, t)
    return out


def unique_with_scale(draws, w, W, s):
    """Ascending unique positions, multiplicities, probabilities and merge scales."""
    uniq, counts = np.unique(draws, return_counts=True)
    p = np.array([int(w[j]) / W for j in uniq.tolist()])
    omega = np.sqrt(counts / (s * p))
    return uniq, counts, p, omega


# ---------------------------------------------------------------------------
# Algorithms 1 and 2: independence loop
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Basis:
    """R (actual fibers as dense columns) and an orthonormal basis of span(R).

    `Ub`, when tracked, is Algorithm 1's literal bordered-inverse update of U.
    It equals (R^T R)^{-1} in exact arithmetic but drifts from it (and can
    overflow) once R is ill-conditioned, so it is kept only for the
    cross-check on well-conditioned inputs; U itself is taken from its
    definition by `inverse_gram`.
    """
    R: np.ndarray          # I_alpha x cap
    Qb: np.ndarray         # I_alpha x cap, orthonormal columns spanning span(R[:, :k])
    k: int                 # number of columns in use
    Ub: np.ndarray | None = None   # cap x cap bordered-update U, if tracked

    @staticmethod
    def empty(n_rows, cap, bordered=False):
        return Basis(np.zeros((n_rows, cap)), np.zeros((n_rows, cap)), 0,
                     np.zeros((cap, cap)) if bordered else None)

    def grow(self, extra):
        cap = self.R.shape[1]
        if self.k + extra <= cap:
            return
        new_cap = max(2 * cap, self.k + extra)
        R = np.zeros((self.R.shape[0], new_cap))
        R[:, :self.k] = self.R[:, :self.k]
        Qb = np.zeros((self.R.shape[0], new_cap))
        Qb[:, :self.k] = self.Qb[:, :self.k]
        if self.Ub is not None:
            Ub = np.zeros((new_cap, new_cap))
            Ub[:self.k, :self.k] = self.Ub[:self.k, :self.k]
            self.Ub = Ub
        self.R, self.Qb = R, Qb


def inverse_gram(R) -> np.ndarray:
    """U = (R^T R)^{-1}, the definition in the proof of Lemma 2.

    Taken from the singular value decomposition R = W S V^T as V S^-2 V^T, an
    algebra that shares nothing with the basis the independence test uses.
    """
    if R.shape[1] == 0:
        return np.zeros((0, 0))
    _, sv, Vt = np.linalg.svd(R, full_matrices=False)
    return (Vt.T / (sv * sv)) @ Vt


def residual_against_span(Qb, x):
    """x minus its orthogonal projection onto span(Qb) (projected twice).

    This is the residual of Algorithm 1's test: with U = (R^T R)^{-1},
    R U R^T is the orthogonal projector onto span(R).  Evaluating it through
    the incrementally updated U loses all accuracy once R is ill-conditioned,
    so the projection is taken with an orthonormal basis of span(R) instead.
    """
    res = x - Qb @ (Qb.T @ x)
    return res - Qb @ (Qb.T @ res)


def independence_loop(basis: Basis, candidates, eps):
    """Visit candidate fibers in order; keep those independent of span(R).

    `candidates` yields dense I_alpha vectors.  Returns (kept flags,
    rho = ||res||^2 / ||x||^2 for every candidate).  A fresh basis (k == 0)
    takes the first candidate unconditionally (Algorithm 1).  Kept
    fibers extend R; if the basis tracks it, also the literal
    bordered-inverse update of U from Algorithm 1.
    """
    kept, rho = [], []
    for x in candidates:
        xx = float(x @ x)
        k = basis.k
        if k == 0:
            basis.grow(1)
            basis.R[:, 0] = x
            if basis.Ub is not None:
                basis.Ub[0, 0] = 1.0 / xx
            basis.Qb[:, 0] = x / math.sqrt(xx)
            basis.k = 1
            kept.append(True)
            rho.append(1.0)
            continue
        res = residual_against_span(basis.Qb[:, :k], x)
        nres = float(np.linalg.norm(res))
        rho.append(nres * nres / xx)
        if nres <= eps * math.sqrt(xx):
            kept.append(False)
            continue
        basis.grow(1)
        if basis.Ub is not None:
            # Algorithm 1's bordered update with delta = ||res||^2, y = U R^T x
            delta = nres * nres
            U = basis.Ub[:k, :k].copy()
            y = U @ (basis.R[:, :k].T @ x)
            basis.Ub[:k, :k] = U + np.outer(y, y) / delta
            basis.Ub[:k, k] = -y / delta
            basis.Ub[k, :k] = -y / delta
            basis.Ub[k, k] = 1.0 / delta
        basis.R[:, k] = x
        basis.Qb[:, k] = res / nres
        basis.k = k + 1
        kept.append(True)
    return kept, rho


# ---------------------------------------------------------------------------
# Algorithm 1 (final step) and Eq. 14: C and the relative error
# ---------------------------------------------------------------------------

def core_matrix(R, u: Unfolding) -> np.ndarray:
    """C_(alpha) = R^T X_(alpha) over the non-empty columns (dense)."""
    return np.asarray((u.mat.T @ R).T)


def error_literal(R, U, C, u: Unfolding) -> float:
    """||X_(alpha) - R U C_(alpha)||_F^2 with X_(alpha) densified (small inputs)."""
    X = u.mat.toarray()
    D = X - R @ (U @ C)
    return float(np.sum(D * D))


def error_projection(R, u: Unfolding, chunk=65536):
    """||X - P X||_F^2 with P the orthogonal projector onto span(R).

    A second algebra for the same quantity: an orthonormal basis from a
    Householder QR of R, then ||X||^2 - sum_f ||Qr^T x_f||^2.  Returns
    (E, per-fiber projected squared norms).
    """
    Qr, _ = np.linalg.qr(R)
    proj = np.empty(u.n_f)
    XT = u.mat.T.tocsr()
    for a in range(0, u.n_f, chunk):
        b = min(u.n_f, a + chunk)
        Z = XT[a:b] @ Qr
        proj[a:b] = np.sum(Z * Z, axis=1)
    return u.norm2 - math.fsum(proj.tolist()), proj


def lstsq_error(R0, u: Unfolding) -> float:
    """Lemma 2: min_L ||X_(alpha) - R0 L||_F^2 via numpy's least squares."""
    X = u.mat.toarray()
    L, *_ = np.linalg.lstsq(R0, X, rcond=None)
    D = X - R0 @ L
    return float(np.sum(D * D))


# ---------------------------------------------------------------------------
# CTD-S (Algorithm 1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class StaticResult:
    unfolding: Unfolding
    draws: np.ndarray        # fiber ids (columns of X_(alpha)) in draw order
    uniq: np.ndarray         # ascending unique fiber ids
    counts: np.ndarray
    p: np.ndarray
    omega: np.ndarray
    accepted: np.ndarray     # fiber ids kept in R, in order of acceptance (ascending)
    rho: np.ndarray          # per unique candidate, ||res||^2/||x||^2
    R: np.ndarray            # I_alpha x s~
    U: np.ndarray            # s~ x s~, (R^T R)^{-1} from its definition
    C: np.ndarray | None     # s~ x n_f, if requested
    err2: float              # ||X - X~||_F^2
    norm2: float             # ||X||_F^2
    proj: np.ndarray | None  # per non-empty fiber ||P x_f||^2 (projection algebra)
    Qb: np.ndarray | None = None  # orthonormal basis of span(R)
    U_bordered: np.ndarray | None = None  # Algorithm 1's literal update of U, if tracked

    @property
    def rel_err(self):
        return self.err2 / self.norm2


def ctd_s_given(u: Unfolding, draw_pos, eps=1e-6, want_C=False, residual="auto",
                w=None, W=None, s=None, bordered=False):
    """CTD-S from given draws (positions into u.fids; duplicates allowed).

    The error is ||X - X~||_F^2 with X~ = R U C_(alpha), which by Lemma 2
    (Eq. 7) is the orthogonal projection of X_(alpha) onto span(R).  The
    default ("projection") evaluates it with a Householder QR of R, which
    stays accurate when R is ill-conditioned; "literal" multiplies out
    R U C with U = (R^T R)^{-1} (small, well-conditioned inputs only).
    `bordered` also tracks Algorithm 1's literal update of U (U_bordered).
    """
    draw_pos = np.asarray(draw_pos, dtype=np.int64)
    s = draw_pos.shape[0] if s is None else s
    if w is None:
        w, W = quantized_weights(u)
    uniq, counts, p, omega = unique_with_scale(draw_pos, w, W, s)
    basis = Basis.empty(u.n_rows, max(1, min(uniq.shape[0], u.n_rows) + 1), bordered)
    kept, rho = independence_loop(basis, (u.column(j) for j in uniq.tolist()), eps)
    kept = np.array(kept, dtype=bool)
    R = basis.R[:, :basis.k].copy()
    U = inverse_gram(R)
    Qb = basis.Qb[:, :basis.k].copy()
    C = core_matrix(R, u) if want_C else None
    if residual == "auto":
        residual = "projection"
    proj = None
    if residual == "literal":
        Cm = C if C is not None else core_matrix(R, u)
        err2 = error_literal(R, U, Cm, u)
    else:
        err2, proj = error_projection(R, u)
    Ub = basis.Ub[:basis.k, :basis.k].copy() if bordered else None
    return StaticResult(u, u.fids[draw_pos], u.fids[uniq], counts, p, omega,
                        u.fids[uniq[kept]], np.array(rho), R, U, C, err2, u.norm2, proj, Qb, Ub)


def ctd_s(dims, idx, val, mode, s, seed, eps=1e-6, want_C=False, residual="auto", tensor=0,
          bordered=False):
    """Algorithm 1 end to end with the Philox draw specification above.

    `tensor` is the counter word that tells the tensors of one batched call
    apart (0 for a single decomposition, b for the b-th tensor of a batch).
    """
    u = unfold(dims, idx, val, mode)
    if not 1 <= s <= u.n_cols_total:
        raise ValueError("sample size out of range")
    w, W = quantized_weights(u)
    draw_pos = sample_columns(w, W, s, seed, step=0, tensor=tensor)
    return ctd_s_given(u, draw_pos, eps, want_C, residual, w=w, W=W, s=s, bordered=bordered)


# ---------------------------------------------------------------------------
# CTD-D (Algorithm 2)
# ---------------------------------------------------------------------------

class Dynamic:
    """CTD-D state: R^(t), U^(t), C^(t)_(alpha), the error and the stream position.

    The time mode is the last mode.  A slice has the first N-1 mode lengths
    of the tensor and length 1 in the time mode; its fiber j becomes column
    j + T * dN_alpha of the grown matricization, T being the number of time
    steps already held.

    With keep_C=False the block update of C is not carried (long streams
    whose C would not fit); `core_columns` still gives any column of C from
    its closed form.
    """

    def __init__(self, dims, idx, val, mode, s, seed, eps=1e-6, keep_dense=False,
                 draw_pos=None, keep_C=True):
        if mode == len(dims) - 1:
            raise ValueError("mode must not be the time mode")
        if keep_dense and not keep_C:
            raise ValueError("the literal error needs C")
        if draw_pos is None:
            st = ctd_s(dims, idx, val, mode, s, seed, eps, want_C=keep_C)
        else:
            st = ctd_s_given(unfold(dims, idx, val, mode), draw_pos, eps, want_C=keep_C)
        self.dims = tuple(int(d) for d in dims)
        self.mode, self.seed, self.eps = mode, seed, eps
        self.static = st
        self.T = self.dims[-1]
        self.dN = st.unfolding.n_cols_total // self.T
        self.basis = Basis.empty(st.R.shape[0], st.R.shape[1] + 64)
        self.basis.R[:, :st.R.shape[1]] = st.R
        self.basis.Qb[:, :st.R.shape[1]] = st.Qb
        self.basis.k = st.R.shape[1]
        self.accepted = list(st.accepted.tolist())
        self.keep_C = keep_C
        self.C = st.C
        self.col_fids = st.unfolding.fids.copy()
        # every input with the size of R right after it was taken in
        self.inputs = [(st.R.shape[1], st.unfolding)]
        self.err2 = st.err2
        self.norm2 = st.norm2
        self.step = 0
        self.X = st.unfolding.mat.toarray() if keep_dense else None
        self.history = []

    @property
    def R(self):
        return self.basis.R[:, :self.basis.k]

    @property
    def U(self):
        """U^(t) = (R^(t)T R^(t))^{-1} (proof of Lemma 2)."""
        return inverse_gram(self.R)

    def core_columns(self, cols) -> np.ndarray:
        """Columns `cols` of C^(t)_(alpha) from their closed form.

        Unrolling Eqs. 8-13: a fiber x taken in at step tau gets the column
        R^(tau)T x, R^(tau) being R right after that step; a later step that
        adds the fibers dR appends dR^T R U C = dR^T P_tau x to it, P_tau the
        orthogonal projector onto span(R^(tau)), because span(R) only grows.
        Since R^(tau)T x = R^(tau)T P_tau x, the column is R^(t)T P_tau x.
        P_tau is taken from a Householder QR of R^(tau).
        """
        cols = np.asarray(cols, dtype=np.int64)
        out = np.zeros((self.basis.k, cols.shape[0]))
        start = 0
        for k_tau, u in self.inputs:
            sel = np.nonzero((cols >= start) & (cols < start + u.n_f))[0]
            if sel.shape[0]:
                Qt, _ = np.linalg.qr(self.R[:, :k_tau])
                Xs = u.mat[:, cols[sel] - start].toarray()
                out[:, sel] = self.R.T @ (Qt @ (Qt.T @ Xs))
            start += u.n_f
        return out

    def update(self, sdims, sidx, sval, d, draw_pos=None):
        """Algorithm 2 on one slice; returns a dict describing the step.

        Draws use Philox counter word `step` = t, the number of this update
        (1 for the first slice); `draw_pos` overrides them with given
        positions into the slice's non-empty fibers.
        """
        if tuple(int(x) for x in sdims) != self.dims[:-1] + (1,):
            raise ValueError("slice shape mismatch")
        u = unfold(sdims, sidx, sval, self.mode)
        if not 1 <= d <= u.n_cols_total:
            raise ValueError("sample size out of range")
        self.step += 1
        k_old = self.basis.k
        R_old = self.R.copy()
        if u.norm2 == 0.0 or u.n_f == 0:
            draws = np.zeros(0, np.int64)
            uniq = np.zeros(0, np.int64)
            kept = np.zeros(0, bool)
            rho = []
        else:
            w, W = quantized_weights(u)
            if draw_pos is None:
                draws = sample_columns(w, W, d, self.seed, step=self.step, tensor=0)
            else:
                draws = np.asarray(draw_pos, dtype=np.int64)
            uniq, counts, p, omega = unique_with_scale(draws, w, W, d)
            kept, rho = independence_loop(self.basis, (u.column(j) for j in uniq.tolist()),
                                          self.eps)
            kept = np.array(kept, dtype=bool)
        dR = self.R[:, k_old:]
        dX = u.mat
        U_old = None
        if self.keep_C:
            # Eq. 13: block update, cross term parenthesized from the left
            top_new = np.asarray((dX.T @ R_old).T)              # R^(t)T dX
            if dR.shape[1]:
                U_old = inverse_gram(R_old)                     # U^(t)
                cross = ((dR.T @ R_old) @ U_old) @ self.C       # ((dR^T R) U) C
                bot_new = np.asarray((dX.T @ dR).T)             # dR^T dX
                self.C = np.block([[self.C, top_new], [cross, bot_new]])
            else:
                self.C = np.hstack([self.C, top_new])
        offset = self.T * self.dN
        new_fids = u.fids + offset
        self.col_fids = np.concatenate([self.col_fids, new_fids])
        self.T += 1
        self.norm2 += u.norm2
        self.accepted.extend((new_fids[uniq[kept]]).tolist() if len(uniq) else [])
        self.inputs.append((self.basis.k, u))
        if self.keep_C and U_old is None:
            U_old = inverse_gram(R_old)
        self.last_blocks = dict(R_old=R_old, U_old=U_old, dR=dR.copy(), dX=dX)
        if self.X is not None:
            self.X = np.hstack([self.X, dX.toarray()])
            D = self.X - self.R @ (self.U @ self.C)
            self.err2 = float(np.sum(D * D))
        else:
            # derived from Eqs. 10-13: the reconstruction of earlier columns is
            # unchanged by a step, and new columns are projected onto span(R^(t+1))
            Qr, _ = np.linalg.qr(self.R)
            Z = dX.T @ Qr
            self.err2 += u.norm2 - math.fsum(np.sum(Z * Z, axis=1).tolist())
        info = dict(step=self.step, draws=u.fids[draws] + offset if len(draws) else draws,
                    uniq=u.fids[uniq] + offset if len(uniq) else uniq,
                    kept=kept, rho=np.array(rho), d_tilde=self.basis.k,
                    added=self.basis.k - k_old, err2=self.err2, norm2=self.norm2,
                    n_cols=self.col_fids.shape[0])
        self.history.append(info)
        return info

    @property
    def rel_err(self):
        return self.err2 / self.norm2

"""Pins of the oracle's U and of its independence residual on inputs shaped like
the paper's workloads.

U is defined as (R^T R)^{-1} (proof of Lemma 2); the oracle takes it from an
SVD of R.  The residual of Algorithm 1's test, rho = ||res||^2 / ||x||^2, is
taken by the oracle from an orthonormal basis built by Gram-Schmidt.  Both are
checked here against algebra that shares nothing with them: the textbook
least-squares residual of a Householder QR (LAPACK geqrf/ormqr), numpy's QR
projector, and the closed-form accuracy of an inverse, on the five
Table-3-shaped tensors, the initial tensor of the CTD-D stream and the stored
oracle run on the 5M-nonzero traffic tensor.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ctd
from workloads import synth

pytestmark = pytest.mark.filterwarnings("error::RuntimeWarning")

U64 = 2.0 ** -52
EPS = 1e-6
BAND = 1e3          # decisions with rho within a factor BAND of eps^2 are not compared
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def householder_rho(u, cand_pos, kept_mask):
    """rho of every candidate against the kept candidates before it (in order).

    A = QR over the kept columns in order (Householder, LAPACK geqrf).  The
    least-squares residual of x against the first m columns of A is the part
    of Q^T x below row m, so rho = sum_{i >= m} (Q^T x)_i^2 / ||x||^2 with m the
    number of kept candidates before x.
    """
    X = np.stack([u.column(j) for j in cand_pos], axis=1)
    K = X[:, kept_mask]
    (h, tau), _ = sla.qr(K, mode="raw")
    ormqr = sla.lapack.get_lapack_funcs("ormqr", (h,))
    lwork = max(1, X.shape[1]) * 64
    qtx, _, info = ormqr("L", "T", h, tau, X.copy(order="F"), lwork)
    assert info == 0
    m_before = np.concatenate([[0], np.cumsum(kept_mask)[:-1]])
    xx = np.einsum("ij,ij->j", X, X)
    rho = np.array([float(qtx[m:, j] @ qtx[m:, j]) for j, m in enumerate(m_before)]) / xx
    return rho


def check_decisions(rho_ora, rho_ref, kept_mask):
    # values: 1e-9 relative (the QR residual of an ill-conditioned kept set carries
    # ~u cond(R_S) relative error), with an absolute floor of 1% of eps^2
    tol = 1e-9 * rho_ref + 1e-2 * EPS * EPS
    assert np.all(np.abs(rho_ora - rho_ref) <= tol), np.max(np.abs(rho_ora - rho_ref) / tol)
    clear = (rho_ref <= EPS * EPS / BAND) | (rho_ref >= EPS * EPS * BAND)
    clear[0] = True
    decide = rho_ref > EPS * EPS
    decide[0] = True               # Algorithm 1 starts R from the first unique fiber
    assert np.array_equal(decide[clear], kept_mask[clear])


def _table3():
    return synth.small_shapes()


@pytest.fixture(scope="module")
def table3_runs():
    out = []
    for t in _table3():
        out.append((t, ctd.ctd_s(t.dims, t.idx, t.val, 0, 300, 7)))
    return out


@pytest.mark.parametrize("i", range(5))
def test_U_is_the_inverse_gram_on_table3_shapes(table3_runs, i):
    """U finite; ||U G - I|| within u cond(G) s~ where that bound is below 1; R U R^T
    equal to the projector of numpy's QR within u cond(R)^2 sqrt(s~) where that bound
    is below 1."""
    _, r = table3_runs[i]
    R, U = r.R, r.U
    k = R.shape[1]
    assert np.all(np.isfinite(U))
    assert np.allclose(U, U.T, rtol=0, atol=1e-12 * np.abs(U).max())
    G = R.T @ R
    sv = np.linalg.svd(R, compute_uv=False)
    cond_R = sv[0] / sv[-1]
    bound_U = U64 * cond_R ** 2 * k
    if bound_U < 1:
        assert np.linalg.norm(U @ G - np.eye(k)) <= bound_U
    Qh, _ = np.linalg.qr(R)
    bound_P = U64 * cond_R ** 2 * np.sqrt(k)
    if bound_P < 1:
        assert np.linalg.norm(R @ U @ R.T - Qh @ Qh.T) <= bound_P


@pytest.mark.parametrize("i", range(5))
def test_independence_residual_equals_least_squares_on_table3_shapes(table3_runs, i):
    t, r = table3_runs[i]
    u = r.unfolding
    pos = np.searchsorted(u.fids, r.uniq)
    kept = np.isin(r.uniq, r.accepted)
    rho = householder_rho(u, pos, kept)
    check_decisions(r.rho, rho, kept)


def test_bordered_update_matches_definition_when_well_conditioned():
    """Algorithm 1's literal bordered update of U agrees with (R^T R)^{-1} to
    u cond(G) s~ where G = R^T R is well conditioned (here cond(G) ~ 1e7)."""
    for t in (_table3()[0], _table3()[3]):
        r = ctd.ctd_s(t.dims, t.idx, t.val, 0, 300, 7, bordered=True)
        k = r.R.shape[1]
        G = r.R.T @ r.R
        cond_G = np.linalg.cond(G)
        assert cond_G < 1e8
        bound = U64 * cond_G * k
        assert np.linalg.norm(r.U_bordered @ G - np.eye(k)) <= bound
        assert np.linalg.norm(r.U_bordered - r.U) <= bound * np.linalg.norm(r.U)


def test_U_and_residual_on_stream_initial_tensor():
    """The 4,000 x 4,000 x 200 initial tensor of the CTD-D stream, s = 800."""
    X = synth.power_law_tensor((4000, 4000, 200), 1_000_000, 4, zipf_a=1.1)  # the stream's initial tensor
    r = ctd.ctd_s(X.dims, X.idx, X.val, 0, 800, 0)
    assert np.all(np.isfinite(r.U))
    u = r.unfolding
    kept = np.isin(r.uniq, r.accepted)
    rho = householder_rho(u, np.searchsorted(u.fids, r.uniq), kept)
    check_decisions(r.rho, rho, kept)
    k = r.R.shape[1]
    sv = np.linalg.svd(r.R, compute_uv=False)
    bound = U64 * (sv[0] / sv[-1]) ** 2 * k
    if bound < 1:
        assert np.linalg.norm(r.U @ (r.R.T @ r.R) - np.eye(k)) <= bound


def test_stored_5m_residuals_equal_least_squares():
    """The stored oracle run on the 5M-nonzero traffic tensor (s = 2000): every
    candidate's rho against the Householder least-squares residual, and the kept
    set against the decisions it implies."""
    g = np.load(os.path.join(GOLDEN, "traffic_5m_s2000_seed0.npz"), allow_pickle=False)
    X = synth.traffic_5m()
    u = ctd.unfold(X.dims, X.idx, X.val, 0)
    uniq = g["unique"].astype(np.int64)
    kept = np.isin(uniq, g["accepted"].astype(np.int64))
    rho = householder_rho(u, np.searchsorted(u.fids, uniq), kept)
    check_decisions(g["rho"], rho, kept)

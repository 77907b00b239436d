"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test ties one part of the oracle to the paper's statements, to closed
forms, to a library routine the method reduces to, or to brute force, so a
plausible slip (dropped term, wrong index or sign, transposed operand) fails.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ctd
from oracle.philox import draw_u128
from workloads import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.filterwarnings("error::RuntimeWarning")


def _dense(t):
    X = np.zeros(t.dims)
    X[tuple(t.idx.astype(np.int64))] = t.val
    return X


def _small(seed=7, dims=(30, 25, 12), nnz=900):
    return synth.uniform_tensor(dims, nnz, seed)


# --- Section 2.1: matricization and the n-mode product (Eqs. 2-3) ----------

@pytest.mark.parametrize("mode", [0, 1, 2])
def test_matricization_matches_textbook_unfolding(mode):
    t = _small()
    u = ctd.unfold(t.dims, t.idx, t.val, mode)
    X = _dense(t)
    # textbook unfolding: mode-n index to rows, the rest column-major (Fortran order)
    Xn = np.reshape(np.moveaxis(X, mode, 0), (t.dims[mode], -1), order="F")
    full = np.zeros_like(Xn)
    full[:, u.fids] = u.mat.toarray()
    assert np.array_equal(full, Xn)
    assert u.norm2 == pytest.approx(float(np.sum(X * X)), rel=1e-15)


def test_n_mode_product_reconstruction():
    """X~ = C x_alpha (R U) elementwise (Eq. 2) equals R U C_(alpha) (Eq. 3)."""
    t = _small(seed=9)
    mode = 0
    r = ctd.ctd_s(t.dims, t.idx, t.val, mode, 40, seed=3, want_C=True)
    I, J, K = t.dims
    s_t = r.R.shape[1]
    Cfull = np.zeros((s_t, J * K))
    Cfull[:, r.unfolding.fids] = r.C
    Ctensor = np.reshape(Cfull, (s_t, J, K), order="F")
    RU = r.R @ r.U
    Xt = np.einsum("ic,cjk->ijk", RU, Ctensor)
    Xunf = np.reshape(Xt, (I, J * K), order="F")
    assert np.allclose(Xunf[:, r.unfolding.fids], RU @ r.C, rtol=1e-12, atol=1e-12)
    X = _dense(t)
    err = float(np.sum((X - Xt) ** 2))
    assert err == pytest.approx(r.err2, rel=1e-9)


def test_matricization_rejects_bad_input():
    t = _small()
    bad = t.idx.copy()
    bad[0, 0] = t.dims[0]
    with pytest.raises(ValueError):
        ctd.unfold(t.dims, bad, t.val, 0)
    dup = np.concatenate([t.idx, t.idx[:, :1]], axis=1)
    with pytest.raises(ValueError):
        ctd.unfold(t.dims, dup, np.concatenate([t.val, t.val[:1]]), 0)
    v = t.val.copy()
    v[3] = np.nan
    with pytest.raises(ValueError):
        ctd.unfold(t.dims, t.idx, v, 0)
    u = ctd.unfold(t.dims, t.idx, np.zeros_like(t.val), 0)
    with pytest.raises(ValueError):
        ctd.quantized_weights(u)
    with pytest.raises(ValueError):
        ctd.ctd_s(t.dims, t.idx, t.val, 0, 0, 0)
    with pytest.raises(ValueError):
        ctd.ctd_s(t.dims, t.idx, t.val, 0, t.dims[1] * t.dims[2] + 1, 0)


# --- Algorithm 1: column distribution and sampling -------------------------

def test_quantized_weights_exact_bound():
    """Each fiber weight is within nnz_f of ||x_f||^2 * 2^sigma (exact rationals)."""
    t = synth.power_law_tensor((40, 30, 10), 2000, 5, zipf_a=1.2)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    v2 = [Fraction(x) ** 2 for x in u.mat.data.tolist()]
    vmax = max(v2)
    e = math.frexp(float(vmax))[1]
    assert Fraction(2) ** (e - 1) <= vmax < Fraction(2) ** e
    sigma = 62 - (len(v2) - 1).bit_length() - e
    assert W < 2 ** 62
    assert W == sum(int(x) for x in w.tolist())
    for j in range(u.n_f):
        a, b = u.mat.indptr[j], u.mat.indptr[j + 1]
        exact = sum(v2[a:b]) * Fraction(2) ** sigma
        assert exact - (b - a) < int(w[j]) <= exact


def test_draw_target_closed_forms():
    """t = floor(r W / 2^128) hits the first and last positive-weight column at the extremes."""
    w = np.array([0, 5, 0, 3, 7, 0], dtype=np.uint64)
    W = 15
    cdf = np.cumsum(w.astype(np.int64))
    for r, expect in ((0, 1), ((1 << 128) - 1, 4)):
        t = (r * W) >> 128
        assert int(np.searchsorted(cdf, t, side="right")) == expect
    # boundaries between columns: target t lands in column j iff cdf[j-1] <= t < cdf[j]
    for t, expect in ((4, 1), (5, 3), (7, 3), (8, 4), (14, 4)):
        assert int(np.searchsorted(cdf, t, side="right")) == expect


def test_sampler_frequencies_match_exact_distribution():
    """Brute force: draw frequencies over many counters against P(i) (chi-square)."""
    t = synth.uniform_tensor((6, 4, 2), 20, 3)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    n = 40000
    pos = ctd.sample_columns(w, W, n, seed=12345)
    obs = np.bincount(pos, minlength=u.n_f)
    col_norm2 = np.asarray(u.mat.multiply(u.mat).sum(axis=0)).ravel()
    p = col_norm2 / col_norm2.sum()
    exp = n * p
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    dof = u.n_f - 1
    # p-value 1e-4 bound via Wilson-Hilferty
    z = 3.72
    bound = dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3
    assert chi2 < bound, (chi2, bound)


def test_zero_weight_columns_never_drawn():
    w = np.array([0, 3, 0, 0, 9, 0], dtype=np.uint64)
    pos = ctd.sample_columns(w, 12, 2000, seed=1)
    assert set(np.unique(pos).tolist()) <= {1, 4}


# --- Algorithm 1 unique selection and the duplicate-merge scale ------------

def _cols(u, positions):
    return np.stack([u.column(j) for j in positions], axis=1)


def test_merge_scale_preserves_outer_product_sum():
    t = synth.power_law_tensor((30, 20, 8), 600, 8, zipf_a=1.2)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    s = 60
    pos = ctd.sample_columns(w, W, s, seed=4)
    uniq, counts, p, omega = ctd.unique_with_scale(pos, w, W, s)
    assert np.array_equal(uniq, np.unique(pos))
    assert counts.sum() == s
    D = _cols(u, pos)
    pw = np.array([int(w[j]) / W for j in pos.tolist()])
    lhs = (D / (s * pw)) @ D.T
    Rp = _cols(u, uniq)
    rhs = (Rp * omega ** 2) @ Rp.T
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())


def test_merged_estimator_is_unbiased():
    """mean over seeds of R' Omega^2 R'^T approaches X_(alpha) X_(alpha)^T."""
    t = synth.uniform_tensor((5, 4, 3), 25, 21)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    s, n_rep = 8, 3000
    acc = []
    for rep in range(n_rep):
        pos = ctd.sample_columns(w, W, s, seed=1000 + rep)
        uniq, counts, p, omega = ctd.unique_with_scale(pos, w, W, s)
        Rp = _cols(u, uniq)
        acc.append(((Rp * omega ** 2) @ Rp.T).ravel())
    acc = np.array(acc)
    mean = acc.mean(axis=0)
    se = acc.std(axis=0) / math.sqrt(n_rep)
    X = u.mat.toarray()
    target = (X @ X.T).ravel()
    assert np.all(np.abs(mean - target) <= 5 * se + 1e-12)


def test_column_scaling_leaves_error_unchanged():
    t = _small(seed=13)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    pos = ctd.sample_columns(w, W, 30, seed=2)
    uniq, counts, p, omega = ctd.unique_with_scale(pos, w, W, 30)
    R = _cols(u, uniq)
    e1 = ctd.lstsq_error(R, u)
    e2 = ctd.lstsq_error(R * omega, u)
    assert e1 == pytest.approx(e2, rel=1e-10)


# --- Algorithm 1 independence loop and Lemma 2 ----------------------------

@pytest.mark.parametrize("seed,s", [(0, 10), (1, 40), (2, 120)])
def test_lemma2_error_equals_least_squares(seed, s):
    t = _small(seed=17 + seed)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    pos = ctd.sample_columns(w, W, s, seed=seed)
    r = ctd.ctd_s_given(u, pos, w=w, W=W, s=s, residual="literal")
    R0 = _cols(u, pos)                     # with duplicates, in draw order
    e_ls = ctd.lstsq_error(R0, u)
    assert r.err2 == pytest.approx(e_ls, rel=1e-9, abs=1e-12 * u.norm2)
    rp = ctd.ctd_s_given(u, pos, w=w, W=W, s=s)
    assert rp.err2 == pytest.approx(e_ls, rel=1e-9, abs=1e-12 * u.norm2)


@pytest.mark.parametrize("dims,nnz,s", [((50, 40, 10), 3000, 80), ((300, 40, 10), 3000, 80)])
def test_U_is_inverse_gram_and_R_holds_actual_fibers(dims, nnz, s):
    t = synth.power_law_tensor(dims, nnz, 23, zipf_a=1.2)
    r = ctd.ctd_s(t.dims, t.idx, t.val, 0, s, seed=5)
    k = r.R.shape[1]
    assert k <= dims[0]
    assert np.linalg.matrix_rank(r.R) == k
    G = r.R.T @ r.R
    cond = np.linalg.cond(G)
    assert np.linalg.norm(r.U @ G - np.eye(k)) <= 1e-13 * cond * k
    u = r.unfolding
    pos = np.searchsorted(u.fids, r.accepted)
    assert np.array_equal(r.R, _cols(u, pos))
    # the CTD-S error is the least-squares error (Lemma 2) in this regime as well
    e_lit = ctd.error_literal(r.R, r.U, ctd.core_matrix(r.R, u), u)
    assert e_lit == pytest.approx(r.err2, rel=1e-6, abs=1e-10 * u.norm2)


def test_accepted_set_matches_greedy_rank_scan():
    """Brute force: keep a candidate iff it raises the rank of the kept set."""
    for seed in range(6):
        t = synth.uniform_tensor((8, 5, 4), 30, 40 + seed)
        u = ctd.unfold(t.dims, t.idx, t.val, 0)
        w, W = ctd.quantized_weights(u)
        pos = ctd.sample_columns(w, W, 15, seed=seed)
        r = ctd.ctd_s_given(u, pos, w=w, W=W, s=15)
        kept = []
        for j in np.unique(pos).tolist():
            M = _cols(u, kept + [j])
            if np.linalg.matrix_rank(M, tol=1e-9) == len(kept) + 1:
                kept.append(j)
        assert np.array_equal(u.fids[kept], r.accepted)


def test_residual_zero_when_all_fibers_drawn():
    t = _small(seed=31, dims=(20, 15, 6), nnz=300)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    r = ctd.ctd_s_given(u, np.arange(u.n_f), s=u.n_f, residual="literal")
    assert r.rel_err <= 1e-13
    assert r.R.shape[1] == np.linalg.matrix_rank(u.mat.toarray())


def test_planted_rank_is_recovered_exactly():
    noisy, clean = synth.planted_low_rank(dims=(60, 50, 20), rank=5, seed=3,
                                          factor_nnz=(12, 10, 4))
    r = ctd.ctd_s(clean.dims, clean.idx, clean.val, 0, 200, seed=0)
    assert r.R.shape[1] == 5
    assert r.rel_err <= 1e-12
    rn = ctd.ctd_s(noisy.dims, noisy.idx, noisy.val, 0, 200, seed=0)
    # the noise floor: with X = S + N and span(R) holding the columns of the signal's
    # unfolding S_(alpha), (I - P) X = (I - P) N, so the error is at most ||N||^2
    un = rn.unfolding
    uc = ctd.unfold(clean.dims, clean.idx, clean.val, 0)
    S = np.zeros((un.n_rows, un.n_cols_total))
    S[:, uc.fids] = uc.mat.toarray()
    D = -S
    D[:, un.fids] += un.mat.toarray()
    Qh, _ = np.linalg.qr(rn.R)
    assert np.linalg.norm(S - Qh @ (Qh.T @ S)) <= 1e-12 * np.linalg.norm(S)
    noise_floor = float(np.sum(D * D)) / un.norm2
    assert 0.5e-4 < noise_floor < 2e-4          # ||N|| = 1% of ||S|| by construction
    assert rn.rel_err <= noise_floor * (1 + 1e-9)


def test_figure2_example():
    g = json.load(open(os.path.join(GOLDEN, "figure_examples.json")))["ctd_s"]
    I, J, K = g["dims"]
    idx, val = [], []
    for name, col in g["column_of"].items():
        for i, v in enumerate(g["fibers"][name]):
            if v:
                idx.append((i, col, 0))
                val.append(v)
    idx = np.array(idx).T.astype(np.int32)
    u = ctd.unfold((I, J, K), idx, np.array(val), 0)
    pos = [g["column_of"][n] for n in g["draws"]]
    r = ctd.ctd_s_given(u, pos, s=len(pos))
    assert r.uniq.tolist() == [g["column_of"][n] for n in g["expect_unique"]]
    assert r.counts.tolist() == g["expect_counts"]
    assert r.accepted.tolist() == [g["column_of"][n] for n in g["expect_kept"]]
    assert r.rel_err == pytest.approx(g["expect_rel_err"], abs=1e-15)


def test_draws_use_documented_counter_layout():
    """Draw j of seed S at step t uses counter (j, j>>32, t, tensor) and key (S, S>>32)."""
    from oracle.philox import philox4x32_10
    seed = (7 << 32) | 99
    x = philox4x32_10((5, 0, 3, 2), (99, 7))
    assert draw_u128(seed, 5, 3, 2) == x[0] | (x[1] << 32) | (x[2] << 64) | (x[3] << 96)


def test_batched_tensor_word_selects_independent_draws():
    """The b-th tensor of a batched call draws with counter word 3 = b (word 0 of a
    single call), so equal tensors in one batch get different samples, and tensor 0
    of a batch reproduces the single decomposition."""
    t = synth.power_law_tensor((30, 20, 8), 600, 8, zipf_a=1.2)
    u = ctd.unfold(t.dims, t.idx, t.val, 0)
    w, W = ctd.quantized_weights(u)
    single = ctd.ctd_s(t.dims, t.idx, t.val, 0, 40, 3)
    b0 = ctd.ctd_s(t.dims, t.idx, t.val, 0, 40, 3, tensor=0)
    b5 = ctd.ctd_s(t.dims, t.idx, t.val, 0, 40, 3, tensor=5)
    assert np.array_equal(single.draws, b0.draws)
    assert not np.array_equal(b0.draws, b5.draws)
    want = ctd.sample_columns(w, W, 40, 3, step=0, tensor=5)
    assert np.array_equal(b5.draws, u.fids[want])


# ---------------------------------------------------------------------------
# Attack candidates read off R (Section 5): group by a coordinate, first
# fiber per group, norm strictly above the representatives' mean.
# ---------------------------------------------------------------------------

def test_attack_readout_worked_example():
    """A 5 x 4 x 3 source x destination x time tensor along the source mode:
    fiber (j, k) has id j + 4 k.  Worked by hand."""
    from oracle.anomaly import attack_candidates, group_coordinate
    dims = (5, 4, 3)
    # kept in this order: (dst 1, t 0), (dst 2, t 0), (dst 1, t 2), (dst 3, t 1)
    accepted = [1, 2, 9, 7]
    norms = [2.0, 1.0, 10.0, 6.0]
    # by destination: representatives are positions 0, 1, 3 (position 2 repeats
    # destination 1); mean (2 + 1 + 6) / 3 = 3, so only position 3 is above it
    c, reps, mean = attack_candidates(accepted, norms, dims, 0, 1)
    assert reps == [0, 1, 3] and mean == 3.0 and c == [3]
    # by time: representatives 0 (t 0), 2 (t 2), 3 (t 1); mean (2 + 10 + 6) / 3
    # = 6, and 6 itself is not above it
    c, reps, mean = attack_candidates(accepted, norms, dims, 0, 2)
    assert reps == [0, 2, 3] and mean == 6.0 and c == [2]
    # a stream's time index grows past the initial length and decodes as is
    assert group_coordinate(3 + 4 * 7, dims, 0, 2) == 7
    assert group_coordinate(3 + 4 * 7, dims, 0, 1) == 3
    with pytest.raises(ValueError):
        group_coordinate(5, dims, 0, 0)


def test_attack_readout_invariants():
    from oracle.anomaly import attack_candidates
    rng = np.random.default_rng(3)
    dims = (50, 30, 40)
    accepted = rng.choice(30 * 40, size=200, replace=False).tolist()
    norms = rng.lognormal(0.0, 1.0, 200)
    c, reps, mean = attack_candidates(accepted, norms, dims, 0, 1)
    assert len(reps) == len({f % 30 for f in accepted})
    # a positive common scale changes no decision
    c2, reps2, _ = attack_candidates(accepted, 7.5 * norms, dims, 0, 1)
    assert c2 == c and reps2 == reps
    # equal norms: nothing is above the mean; one group: nothing either
    assert attack_candidates(accepted, np.ones(200), dims, 0, 1)[0] == []
    same_dst = [3 + 30 * k for k in range(10)]
    assert attack_candidates(same_dst, np.arange(1.0, 11.0), dims, 0, 1)[0] == []


def test_attack_readout_finds_injected_attacks():
    """CTD-D with the paper's d = 10, eps = 0.15 on traffic with three injected
    attacks (20 % of the sources each hit one victim): every (victim, time)
    of an attack is among the candidates."""
    from oracle.anomaly import attack_candidates, group_coordinate
    a = synth.attack_stream()
    X = a.initial
    D = ctd.Dynamic(X.dims, X.idx, X.val, 0, 100, 0, eps=0.15)
    for sl in a.slices:
        D.update(sl.dims, sl.idx, sl.val, 10)
    norms = np.sqrt((D.R * D.R).sum(axis=0))
    c, _, _ = attack_candidates(D.accepted, norms, D.dims, 0, 1)
    found = {(group_coordinate(D.accepted[i], D.dims, 0, 1),
              group_coordinate(D.accepted[i], D.dims, 0, 2)) for i in c}
    T0 = X.dims[2]
    for t, victim, _ in a.attacks:
        assert (victim, T0 + t) in found


# ---------------------------------------------------------------------------
# Memory usage of the factors (Eq. 15)
# ---------------------------------------------------------------------------

def test_memory_usage_worked_example():
    """R's fibers a (rows 0, 1), b (rows 1, 2) and c (row 5) on a 6 x 4 matrix
    X: a and b share row 1, so U = (R^T R)^{-1} has a dense 2 x 2 block and a
    1 x 1 block, 5 nonzeros; the inverse computed directly agrees."""
    from oracle.metrics import memory_usage, structural_nnz_U
    R = np.zeros((6, 3))
    R[[0, 1], 0] = [1.0, 2.0]
    R[[1, 2], 1] = [3.0, 1.0]
    R[5, 2] = 4.0
    U = np.linalg.inv(R.T @ R)
    assert structural_nnz_U(R) == 5 == int(np.count_nonzero(np.abs(U) > 1e-12))
    X = np.zeros((6, 4))
    X[0, 0] = 1.0      # meets a only
    X[2, 1] = 1.0      # meets b only
    X[4, 2] = 1.0      # meets nothing: an empty column of C
    X[1, 3] = X[5, 3] = 1.0   # meets a, b and c
    C = R.T @ X
    nc, nu, nr, usage = memory_usage(R, C, int(np.count_nonzero(X)))
    assert (nc, nu, nr) == (1 + 1 + 0 + 3, 5, 5)
    assert usage == (5 + 5 + 5) / 5


def test_structural_U_matches_inverse_on_block_data():
    """Fibers drawn inside disjoint row blocks: the structural count equals the
    nonzeros of the explicitly inverted Gram."""
    from oracle.metrics import structural_nnz_U
    rng = np.random.default_rng(4)
    R = np.zeros((40, 12))
    blocks = [(0, 10, [0, 1, 2, 3]), (10, 25, [4, 5, 6]), (25, 40, [7, 8, 9, 10, 11])]
    for r0, r1, cols in blocks:
        for c in cols:
            rows = rng.choice(np.arange(r0, r1), size=5, replace=False)
            R[rows, c] = rng.random(5) + 0.5
    U = np.linalg.inv(R.T @ R)
    expect = int(np.count_nonzero(np.abs(U) > 1e-12 * np.abs(U).max()))
    assert structural_nnz_U(R) <= 16 + 9 + 25
    assert structural_nnz_U(R) == expect


def test_error_nonincreasing_in_sample_size():
    """Sample-size sweep on the Haggle-shaped tensor of Table 3 (the paper's
    Fig. 5 methodology, mode alpha = 1, s from 1 to 1000).  Draw j depends only
    on its Philox counter, so the draws for s1 < s2 are a prefix of those for
    s2 and the candidate set only grows: the error, the distance of X_(alpha)
    from the span of the kept fibers, cannot grow beyond the epsilon-skips
    (each skipped fiber lies within eps ||x|| of the span).  The kept count is
    bounded by rank X_(alpha), computed here from X X^T."""
    X = synth.small_shapes()[1]
    u = ctd.unfold(X.dims, X.idx, X.val, 0)
    G = (u.mat @ u.mat.T).toarray()
    rank = int(np.linalg.matrix_rank(G, tol=1e-9 * np.abs(G).max()))
    prev_draws, prev_err = None, None
    for s in (1, 5, 20, 100, 400, 1000):
        o = ctd.ctd_s(X.dims, X.idx, X.val, 0, s, 3)
        if prev_draws is not None:
            assert np.array_equal(o.draws[:len(prev_draws)], prev_draws), s
            assert o.rel_err <= prev_err + 1e-9, (s, o.rel_err, prev_err)
        assert len(o.accepted) <= rank, (s, len(o.accepted), rank)
        if len(o.accepted) == rank:   # the kept fibers span the column space
            assert o.rel_err <= 1e-12, (s, o.rel_err)
        prev_draws, prev_err = o.draws, o.rel_err


def test_sparse_core_worked_example():
    """The sparse C of the Eq. 15 worked example, by hand: R's fibers a (rows
    0, 1; values 1, 2), b (rows 1, 2; values 3, 1), c (row 5; value 4);
    X's columns e0, e2, e4 and e1 + e5.  C = R^T X has column 0 = (1, 0, 0),
    column 1 = (0, 1, 0), column 2 empty (row 4 meets no kept fiber) and
    column 3 = (2, 3, 4)."""
    from oracle.metrics import sparse_core
    R = np.zeros((6, 3))
    R[[0, 1], 0] = [1.0, 2.0]
    R[[1, 2], 1] = [3.0, 1.0]
    R[5, 2] = 4.0
    idx = np.array([[0, 2, 4, 1, 5], [0, 1, 2, 3, 3]], dtype=np.int32)
    u = ctd.unfold((6, 4), idx, np.ones(5), 0)
    indptr, indices, data = sparse_core(R, u)
    assert indptr.tolist() == [0, 1, 2, 2, 5]
    assert indices.tolist() == [0, 1, 0, 1, 2]
    assert data.tolist() == [1.0, 1.0, 2.0, 3.0, 4.0]

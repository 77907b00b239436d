"""Pins of the CTD-D oracle (Algorithm 2, Eqs. 8-13)."""
import json
import os

import numpy as np
import pytest

from oracle import ctd
from workloads import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.filterwarnings("error::RuntimeWarning")


def _stream(seed=3, dims=(24, 18, 6), nnz0=500, n_slices=6):
    st = synth.traffic_stream(dims=dims, nnz0=nnz0, n_slices=n_slices,
                              slice_nnz=(40, 120), zipf_a=1.1, n_anomalies=1,
                              block=5, seed=seed)
    return st


def test_block_update_equals_direct_product():
    """C^(t+1) = R^(t+1)T [R^(t) U^(t) C^(t), dX] (Eqs. 9, 12, 13)."""
    st = _stream()
    dyn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 30, seed=2)
    saw_growth = saw_empty = False
    for sl in st.slices:
        C_old = dyn.C.copy()
        dyn.update(sl.dims, sl.idx, sl.val, d=4)
        b = dyn.last_blocks
        direct = dyn.R.T @ np.hstack([b["R_old"] @ b["U_old"] @ C_old, b["dX"].toarray()])
        assert np.allclose(dyn.C, direct, rtol=1e-9, atol=1e-9 * np.abs(direct).max())
        if b["dR"].shape[1]:
            saw_growth = True
        else:
            saw_empty = True
            # empty dR: only new columns are added (Algorithm 2)
            assert dyn.C.shape[0] == C_old.shape[0]
    assert saw_growth


def test_core_columns_closed_form_equals_block_update():
    """Every column of C^(t) from its closed form R^(t)T P_tau x (a QR projector)
    equals the block update of Eq. 13 with U = (R^T R)^{-1}, after every step."""
    st = _stream(seed=13, n_slices=8)
    dyn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 30, seed=3)
    grew = 0
    for sl in st.slices:
        info = dyn.update(sl.dims, sl.idx, sl.val, d=4)
        grew += info["added"] > 0
        ref = dyn.core_columns(np.arange(dyn.C.shape[1]))
        cond = np.linalg.cond(dyn.R)
        tol = max(1e-13, 2.0 ** -52 * cond ** 2 * 10)
        assert np.abs(dyn.C - ref).max() <= tol * np.abs(ref).max()
    assert grew >= 2


def test_empty_delta_R_adds_columns_only():
    st = _stream(seed=5, dims=(8, 18, 6))
    dyn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 100, seed=1)
    sl = st.slices[0]
    # draw a slice fiber that already lies in span(R): reuse a fiber of R itself
    u = ctd.unfold(sl.dims, sl.idx, sl.val, 0)
    C_old = dyn.C.copy()
    k_old = dyn.R.shape[1]
    if k_old < dyn.R.shape[0]:
        pytest.skip("R does not span the row space for this draw")
    dyn.update(sl.dims, sl.idx, sl.val, d=3)
    assert dyn.R.shape[1] == k_old
    assert np.array_equal(dyn.C[:, :C_old.shape[1]], C_old)
    assert np.allclose(dyn.C[:, C_old.shape[1]:], dyn.R.T @ u.mat.toarray())


def test_frozen_history_error_identity():
    """Literal ||X^(t) - R U C||^2 equals E^(t) + ||dX - P dX||^2 step by step."""
    st = _stream(seed=7)
    lit = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 30, seed=4,
                      keep_dense=True)
    idn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 30, seed=4)
    assert lit.err2 == pytest.approx(idn.err2, rel=1e-9)
    for sl in st.slices:
        a = lit.update(sl.dims, sl.idx, sl.val, d=4)
        b = idn.update(sl.dims, sl.idx, sl.val, d=4)
        assert np.array_equal(a["draws"], b["draws"])
        assert a["d_tilde"] == b["d_tilde"]
        assert lit.err2 == pytest.approx(idn.err2, rel=1e-8, abs=1e-12 * lit.norm2)
        assert lit.norm2 == pytest.approx(idn.norm2, rel=1e-14)


def test_slices_draw_with_their_own_step_counter():
    st = _stream(seed=9)
    dyn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 20, seed=6)
    sl = st.slices[0]
    info = dyn.update(sl.dims, sl.idx, sl.val, d=5)
    u = ctd.unfold(sl.dims, sl.idx, sl.val, 0)
    w, W = ctd.quantized_weights(u)
    pos = ctd.sample_columns(w, W, 5, seed=6, step=1)
    T0 = st.initial.dims[-1]
    assert np.array_equal(info["draws"], u.fids[pos] + T0 * st.initial.dims[1])


def test_figure3_example():
    g = json.load(open(os.path.join(GOLDEN, "figure_examples.json")))
    gs, gd = g["ctd_s"], g["ctd_d"]
    I, J, _ = gs["dims"]

    def coo(fibers, column_of, k):
        idx, val = [], []
        for name, col in column_of.items():
            for i, v in enumerate(fibers[name]):
                if v:
                    idx.append((i, col, k))
                    val.append(v)
        return np.array(idx).T.astype(np.int32), np.array(val)

    idx, val = coo(gs["fibers"], gs["column_of"], 0)
    pos = [gs["column_of"][n] for n in gs["draws"]]
    dyn = ctd.Dynamic((I, J, 1), idx, val, 0, len(pos), seed=0, keep_dense=True, draw_pos=pos)
    assert dyn.R.shape[1] == 2
    sidx, sval = coo(gd["slice_fibers"], gd["slice_column_of"], 0)
    cols = [gd["slice_column_of"][n] for n in ("purple", "green2")]
    info = dyn.update((I, J, 1), sidx, sval, d=2, draw_pos=cols)
    kept = [n for n, k in zip(("purple", "green2"), info["kept"]) if k]
    assert kept == gd["expect_kept"]
    assert dyn.R.shape[1] == 3
    assert dyn.rel_err == pytest.approx(0.0, abs=1e-14)


def test_update_rejects_bad_slices():
    st = _stream(seed=11)
    dyn = ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 10, seed=0)
    sl = st.slices[0]
    with pytest.raises(ValueError):
        dyn.update((sl.dims[0], sl.dims[1], 2), sl.idx, sl.val, d=2)
    with pytest.raises(ValueError):
        dyn.update(sl.dims, sl.idx, sl.val, d=0)
    with pytest.raises(ValueError):
        ctd.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 2, 10, seed=0)

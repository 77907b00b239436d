"""Checkpoint and resume of a CTD-D stream (ctd_save_state / ctd_load_state)
through the C ABI: the full-size 4,000 x 4,000 x 200 traffic stream (s = 800,
d = 8) straight through its 200 slices, against the same stream saved after
slice 100, destroyed, and resumed on a new handle.  The resumed run must give
the same draws and kept fibers at every call and the same bits in the error,
R, Q, M and sampled columns of C (Algorithm 2 carries R, U and C between
steps, Section 3.2); the checkpoint must also agree with the stored oracle
results at slice 100."""
import os

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "stream_4000_s800_d8.npz")
SAVE_AT = 100


@pytest.fixture(scope="module")
def stream():
    return synth.traffic_stream()


def _steps(ctd, h, slices, lo, hi, batch):
    out = []
    for t in range(lo, hi, batch):
        if batch == 1:
            h.update(*slices[t], 8)
        else:
            h.update_batched(slices[t:t + batch], 8)
        r = h.result()
        out.append((r["step"], r["draws"], r["accepted"], r["rel_err"], r["err2"], r["norm2"]))
    return out


def _final(h, cols):
    f = h.result(factors=True, core=False)
    return dict(R=f["R"], Q=f["Q"], M=f["Linv_t"], acc=f["accepted"], col=f["col_ids"],
                C=h.core_columns(cols), err2=f["err2"], norm2=f["norm2"], step=f["step"])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,batch", [("fp64", 1), ("mixed", 4)])
def test_resume_from_checkpoint_is_bit_identical(stream, precision, batch):
    import paper_1710_03608_amd as ctd
    ctd.load_library()
    g = np.load(GOLD, allow_pickle=False)
    st = stream
    dims, idx, val = ctd.to_device(st.initial, "cuda")
    slices = [ctd.to_device(sl, "cuda") for sl in st.slices]
    n = len(slices)
    cols = g["C_cols"]

    h = ctd.Ctd(precision=precision, want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 800, 0)
        straight = _steps(ctd, h, slices, 0, n, batch)
        ref = _final(h, cols)
    finally:
        h.close()

    h = ctd.Ctd(precision=precision, want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 800, 0)
        first = _steps(ctd, h, slices, 0, SAVE_AT, batch)
        at_save = h.result()
        buf = h.save_state()
    finally:
        h.close()
    assert at_save["step"] == SAVE_AT
    assert at_save["s_tilde"] == int(g["d_tilde"][SAVE_AT - 1])
    rel = float(g["err2"][SAVE_AT - 1] / g["norm2"][SAVE_AT - 1])
    tol = 1e-6 if precision == "fp64" else 1e-4
    assert abs(at_save["rel_err"] - rel) <= tol * rel + 1e-12

    h = ctd.Ctd(precision=precision, want_C=True)
    try:
        h.load_state(buf)
        del buf
        r = h.result()
        assert r["step"] == SAVE_AT and r["s_tilde"] == at_save["s_tilde"]
        assert r["s"] == 0 and r["s_unique"] == 0
        assert np.array_equal(r["accepted"], at_save["accepted"])
        assert r["err2"] == at_save["err2"] and r["norm2"] == at_save["norm2"]
        assert r["n_cols"] == at_save["n_cols"]
        second = _steps(ctd, h, slices, SAVE_AT, n, batch)
        got = _final(h, cols)
    finally:
        h.close()

    resumed = first + second
    assert len(resumed) == len(straight)
    for a, b in zip(straight, resumed):
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]), a[0]
        assert np.array_equal(a[2], b[2]), a[0]
        assert a[3] == b[3] and a[4] == b[4] and a[5] == b[5], a[0]
    assert got["step"] == ref["step"] == n
    for key in ("R", "Q", "M", "acc", "col", "C"):
        assert ref[key].dtype == got[key].dtype and ref[key].shape == got[key].shape, key
        assert np.array_equal(ref[key].view(np.uint8), got[key].view(np.uint8)), key
    assert got["err2"] == ref["err2"] and got["norm2"] == ref["norm2"]
    assert np.array_equal(got["acc"], g["all_accepted"])


def test_state_arguments(stream):
    import paper_1710_03608_amd as ctd
    ctd.load_library()
    X = synth.uniform_tensor((40, 30, 8), 800, 3)
    dims, idx, val = ctd.to_device(X, "cuda")
    h = ctd.Ctd(precision="fp64", want_C=False)
    try:
        h.decompose(dims, idx, val, 0, 20, 1)
        with pytest.raises(ctd.CtdError) as ei:          # no CTD-D stream without C
            h.save_state()
        assert ei.value.name == "CTD_ERR_STATE"
    finally:
        h.close()
    h = ctd.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 20, 1)
        buf = h.save_state()                              # step 0: right after CTD-S
        with pytest.raises(ctd.CtdError) as ei:
            h.load_state(buf[:buf.shape[0] // 2])
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
        bad = buf.copy()
        bad[0] ^= 1
        with pytest.raises(ctd.CtdError) as ei:
            h.load_state(bad)
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
    finally:
        h.close()
    h2 = ctd.Ctd(precision="mixed", want_C=True)
    try:
        with pytest.raises(ctd.CtdError) as ei:           # precision differs
            h2.load_state(buf)
        assert ei.value.name == "CTD_ERR_STATE"
    finally:
        h2.close()
    h3 = ctd.Ctd(precision="fp64", want_C=True)
    try:
        h3.load_state(buf)
        r = h3.result(factors=True)
        assert r["step"] == 0 and r["s_tilde"] > 0
        sl = synth.uniform_tensor((40, 30, 1), 60, 4)
        h3.update(*ctd.to_device(sl, "cuda"), 3)
        assert h3.result()["step"] == 1
    finally:
        h3.close()

"""CTD-D on the GPU (through the C ABI) against the CPU float64 oracle (Algorithm 2)."""
import numpy as np
import pytest

from c_bounds import core_error_bound
from oracle import ctd as ora
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1710_03608_amd as ctd
    assert torch.cuda.is_available()
    ctd.load_library()
    return ctd


def _stream(seed, dims=(60, 50, 12), nnz0=2500, n_slices=8, slice_nnz=(60, 400)):
    return synth.traffic_stream(dims=dims, nnz0=nnz0, n_slices=n_slices, slice_nnz=slice_nnz,
                                zipf_a=1.1, n_anomalies=1, block=6, seed=seed)


def reference_core(st, o):
    """C_(alpha) from its definition: column f holds R^T P_{t_f} x_f, P_{t_f} the
    projector onto span(R) at the step where fiber f arrived (Eqs. 8-13 unrolled)."""
    R = o.R
    k_at = [len(o.static.accepted)] + [h["d_tilde"] for h in o.history]
    inputs = [st.initial] + list(st.slices)
    cols = []
    for t, X in enumerate(inputs):
        u = ora.unfold(X.dims, X.idx, X.val, 0)
        Qt, _ = np.linalg.qr(R[:, :k_at[t]])
        Xd = u.mat.toarray()
        cols.append(R.T @ (Qt @ (Qt.T @ Xd)))
    return np.hstack(cols)


def check_core(st, o, final, batch, precision="fp64"):
    """The GPU's C against its closed form, entry by entry within the running error
    bound of the library's arithmetic (c_bounds.core_error_bound)."""
    ref = reference_core(st, o)
    C = final["C"].astype(np.float64)
    assert C.shape == ref.shape
    ncols = [o.static.unfolding.n_f] + [h["n_cols"] for h in o.history]
    ranks = [len(o.static.accepted)] + [h["d_tilde"] for h in o.history]
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    bound = core_error_bound([st.initial] + list(st.slices), ncols, ranks, np.arange(C.shape[1]),
                             final["R"], final["Q"], final["Linv_t"], ref, batch, u)
    bound += 64 * 2.0 ** -52 * np.abs(ref).max()     # the closed form's own rounding
    assert np.all(np.abs(C - ref) <= bound), np.max(np.abs(C - ref) / bound)


def _run(lib, st, s, d, seed, precision="fp64"):
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(precision=precision, want_C=True)
    h.decompose(dims, idx, val, 0, s, seed)
    steps = [h.result()]
    for sl in st.slices:
        sd, si, sv = lib.to_device(sl, "cuda")
        h.update(sd, si, sv, d)
        steps.append(h.result(factors=False))
    final = h.result(factors=True)
    h.close()
    return steps, final


@pytest.mark.parametrize("seed,s,d,J", [(3, 30, 4, 50), (5, 50, 8, 50), (7, 20, 100, 200)])
def test_stream_matches_oracle(lib, seed, s, d, J):
    st = _stream(seed, dims=(60, J, 12))
    o = ora.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, s, seed)
    steps, final = _run(lib, st, s, d, seed)
    T0, J = st.initial.dims[2], st.initial.dims[1]
    assert np.array_equal(steps[0]["accepted"], o.static.accepted.astype(np.uint64))
    for t, sl in enumerate(st.slices):
        info = o.update(sl.dims, sl.idx, sl.val, d)
        g = steps[t + 1]
        off = (T0 + t) * J
        assert np.array_equal(g["draws"] + np.uint64(off), info["draws"].astype(np.uint64)), t
        assert g["s_tilde"] == info["d_tilde"], t
        assert g["step"] == t + 1
        assert abs(g["rel_err"] - o.rel_err) <= 1e-6 * o.rel_err + 1e-12, (t, g["rel_err"], o.rel_err)
        assert g["norm2"] == pytest.approx(o.norm2, rel=1e-13)
    assert np.array_equal(np.sort(final["accepted"]), np.sort(np.array(o.accepted, dtype=np.uint64)))
    assert np.array_equal(final["col_ids"], o.col_fids.astype(np.uint64))
    R = final["R"]
    assert np.array_equal(R, o.R)
    check_core(st, o, final, 1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_slices_take_the_hot_row_projection(lib, precision):
    """Slices of more than 2^18 nonzeros over 1500 rows: their residual runs
    through the hot-row split of the projection, with Q of the grown basis
    (leading dimension the stream's capacity) and its column count."""
    st = synth.traffic_stream(dims=(1500, 2000, 4), nnz0=300000, n_slices=2,
                              slice_nnz=(280000, 290000), zipf_a=1.1, n_anomalies=0, seed=21)
    assert all(sl.nnz > 2 ** 18 for sl in st.slices)
    o = ora.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 600, 21)
    steps, final = _run(lib, st, 600, 20, 21, precision=precision)
    rtol, atol = (1e-6, 1e-12) if precision == "fp64" else (1e-4, 1e-8)
    assert np.array_equal(steps[0]["accepted"], o.static.accepted.astype(np.uint64))
    for t, sl in enumerate(st.slices):
        info = o.update(sl.dims, sl.idx, sl.val, 20)
        g = steps[t + 1]
        assert g["s_tilde"] == info["d_tilde"], t
        assert abs(g["rel_err"] - o.rel_err) <= rtol * o.rel_err + atol, (t, g["rel_err"], o.rel_err)
    assert np.array_equal(np.sort(final["accepted"]), np.sort(np.array(o.accepted, dtype=np.uint64)))
    check_core(st, o, final, 1, precision)


def test_empty_and_zero_slices(lib):
    import torch
    st = _stream(9, n_slices=2)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(want_C=True)
    h.decompose(dims, idx, val, 0, 20, 1)
    r0 = h.result()
    sd = st.slices[0].dims
    h.update(sd, torch.zeros((3, 0), dtype=torch.int32, device="cuda"),
             torch.zeros(0, dtype=torch.float64, device="cuda"), 2)
    r1 = h.result()
    assert r1["err2"] == r0["err2"] and r1["s_tilde"] == r0["s_tilde"] and r1["step"] == 1
    _, si, sv = lib.to_device(st.slices[1], "cuda")
    h.update(sd, si, torch.zeros_like(sv), 2)
    r2 = h.result()
    assert r2["err2"] == r0["err2"] and r2["s_tilde"] == r0["s_tilde"] and r2["step"] == 2
    h.close()


def test_update_argument_checks(lib):
    st = _stream(11, n_slices=1)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(want_C=True)
    h.decompose(dims, idx, val, 0, 20, 1)
    sd, si, sv = lib.to_device(st.slices[0], "cuda")
    for bad_dims, d, code in (((sd[0], sd[1], 2), 2, "CTD_ERR_STATE"),
                              ((sd[0] + 1, sd[1], 1), 2, "CTD_ERR_STATE"),
                              (sd, 0, "CTD_ERR_INVALID_ARG")):
        with pytest.raises(lib.CtdError) as ei:
            h.update(bad_dims, si, sv, d)
        assert ei.value.name == code
    h.close()
    h2 = lib.Ctd(want_C=False)
    h2.decompose(dims, idx, val, 0, 20, 1)
    with pytest.raises(lib.CtdError) as ei:
        h2.update(sd, si, sv, 2)
    assert ei.value.name == "CTD_ERR_STATE"
    h2.close()


@pytest.mark.parametrize("B", [2, 3, 8])
def test_batched_update_equals_sequential(lib, B):
    """ctd_update_batched over B slices gives what B calls of ctd_update give: the same
    draws and kept fibers, errors to rounding, and C (the rows of the batch's kept
    fibers over earlier columns come from one deferred pass)."""
    st = _stream(5, dims=(60, 50, 12), n_slices=8)
    o = ora.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 50, 5)
    seq_steps, seq_final = _run(lib, st, 50, 8, 5)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 50, 5)
        slices = [lib.to_device(sl, "cuda") for sl in st.slices]
        for i in range(0, len(slices), B):
            h.update_batched(slices[i:i + B], 8)
            r = h.result()
            ref = seq_steps[min(i + B, len(slices))]
            assert r["step"] == ref["step"]
            assert np.array_equal(r["accepted"], ref["accepted"])
            assert abs(r["rel_err"] - ref["rel_err"]) <= 1e-12 * ref["rel_err"] + 1e-15
        final = h.result(factors=True)
    finally:
        h.close()
    assert np.array_equal(final["col_ids"], seq_final["col_ids"])
    assert final["C"].shape == seq_final["C"].shape
    for sl in st.slices:
        o.update(sl.dims, sl.idx, sl.val, 8)
    check_core(st, o, final, B)
    check_core(st, o, seq_final, 1)


def test_batched_update_argument_checks(lib):
    st = _stream(11, n_slices=2)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 20, 1)
        sd, si, sv = lib.to_device(st.slices[0], "cuda")
        with pytest.raises(lib.CtdError) as ei:
            h.update_batched([(sd, si, sv), ((sd[0], sd[1], 2), si, sv)], 2)
        assert ei.value.name == "CTD_ERR_STATE"
        with pytest.raises(lib.CtdError) as ei:
            h.update_batched([], 2)
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
        h.update_batched([(sd, si, sv)], 2)      # the handle is still usable
        assert h.result()["step"] == 1
    finally:
        h.close()


def test_four_way_stream_matches_oracle(lib):
    """CTD-D on a 4-way tensor (time last) along mode 0."""
    X = synth.uniform_tensor((40, 10, 8, 6), 2000, 41)
    slices = [synth.uniform_tensor((40, 10, 8, 1), 150 + 40 * t, 50 + t) for t in range(5)]
    o = ora.Dynamic(X.dims, X.idx, X.val, 0, 25, 3)
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 25, 3)
        for sl in slices:
            o.update(sl.dims, sl.idx, sl.val, 5)
            sd, si, sv = lib.to_device(sl, "cuda")
            h.update(sd, si, sv, 5)
            r = h.result()
            assert np.array_equal(r["accepted"], np.asarray(o.accepted, dtype=np.uint64))
            rel = o.err2 / o.norm2
            assert abs(r["rel_err"] - rel) <= 1e-6 * rel + 1e-12, (r["rel_err"], rel)
    finally:
        h.close()


@pytest.mark.parametrize("B", [1, 4, 8])
def test_mixed_core_held_in_float32(lib, B):
    """A mixed-precision handle holds the CTD-D C in float32 (new columns and the
    cross term on float32 MFMAs; batches of more than 16 new rows on bfloat16
    MFMAs with three-part operands): the same kept fibers as float64, and C
    against its closed form (the oracle's R) within the running error bound of a
    float32 C."""
    st = _stream(5, dims=(60, 50, 12), n_slices=8)
    o = ora.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 50, 5)
    for sl in st.slices:
        o.update(sl.dims, sl.idx, sl.val, 8)
    _, ref = _run(lib, st, 50, 8, 5)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(precision="mixed", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 50, 5)
        slices = [lib.to_device(sl, "cuda") for sl in st.slices]
        for i in range(0, len(slices), B):
            if B == 1:
                h.update(*slices[i], 8)
            else:
                h.update_batched(slices[i:i + B], 8)
        final = h.result(factors=True)
    finally:
        h.close()
    assert final["C"].dtype == np.float32
    assert np.array_equal(final["accepted"], ref["accepted"])
    assert np.array_equal(final["col_ids"], ref["col_ids"])
    assert np.array_equal(final["R"], o.R)
    check_core(st, o, final, B, precision="mixed")

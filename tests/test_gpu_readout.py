"""Attack candidates read off R on the GPU (ctd_attack_candidates) against the
oracle's readout (Section 5), on the GPU's own kept fibers with norms taken
from the input data."""
import numpy as np
import pytest

from oracle import ctd as ora
from oracle.anomaly import attack_candidates, group_coordinate
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1710_03608_amd as ctd
    assert torch.cuda.is_available()
    ctd.load_library()
    return ctd


def fiber_norms(tensors, mode, offsets):
    """||x_f|| of every fiber id of the given inputs (a stream's slices carry
    their column offset), straight from the nonzeros."""
    out = {}
    for X, off in zip(tensors, offsets):
        f = ora.fiber_ids(X.dims, X.idx, mode) + off
        order = np.argsort(f, kind="stable")
        fs, vs = f[order], X.val[order]
        starts = np.flatnonzero(np.r_[True, fs[1:] != fs[:-1]])
        sums = np.add.reduceat(vs * vs, starts)
        for fid, s2 in zip(fs[starts].tolist(), sums.tolist()):
            out[int(fid)] = np.sqrt(s2)
    return out


def check_against_oracle(g, accepted, norm_of, dims, group_mode):
    norms = np.array([norm_of[int(f)] for f in accepted])
    c, reps, _ = attack_candidates(accepted.tolist(), norms, dims, 0, group_mode)
    assert g["n_groups"] == len(reps)
    assert g["count"] == len(c)
    assert np.array_equal(g["fids"], accepted[c])
    np.testing.assert_allclose(g["norms"], norms[c], rtol=1e-12, atol=0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_readout_after_decompose(lib, precision):
    X = synth.power_law_tensor((300, 400, 30), 20000, 9, zipf_a=1.2)
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision=precision)
    try:
        h.decompose(dims, idx, val, 0, 300, 4)
        accepted = h.result()["accepted"]
        norm_of = fiber_norms([X], 0, [0])
        for gm in (1, 2):
            g = h.attack_candidates(gm)
            check_against_oracle(g, accepted, norm_of, X.dims, gm)
        # a small cap returns the first candidates and the full count
        g_all = h.attack_candidates(1)
        g2 = h.attack_candidates(1, cap=2)
        assert g2["count"] == g_all["count"]
        assert np.array_equal(g2["fids"], g_all["fids"][:2])
        with pytest.raises(lib.CtdError):
            h.attack_candidates(0)
        with pytest.raises(lib.CtdError):
            h.attack_candidates(3)
    finally:
        h.close()


def test_readout_finds_injected_attacks_in_stream(lib):
    """CTD-D with the paper's d = 10, eps = 0.15 over traffic with three
    injected attacks: every (victim, time) is a candidate, and the readout
    equals the oracle's on the GPU's kept fibers."""
    a = synth.attack_stream()
    X = a.initial
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True, eps=0.15)
    try:
        h.decompose(dims, idx, val, 0, 100, 0)
        for sl in a.slices:
            sd, si, sv = lib.to_device(sl, "cuda")
            h.update(sd, si, sv, 10)
        accepted = h.result()["accepted"]
        g = h.attack_candidates(1)
    finally:
        h.close()
    I, J, T0 = X.dims
    offsets = [0] + [(T0 + t) * J for t in range(len(a.slices))]
    norm_of = fiber_norms([X] + a.slices, 0, offsets)
    check_against_oracle(g, accepted, norm_of, X.dims, 1)
    found = {(group_coordinate(int(f), X.dims, 0, 1), group_coordinate(int(f), X.dims, 0, 2))
             for f in g["fids"]}
    for t, victim, _ in a.attacks:
        assert (victim, T0 + t) in found


def test_memory_usage_ctd_s(lib):
    """Eq. 15 on the GPU equals the oracle's count from its own R and C
    (same kept fibers in float64; positive values, so no entry of C cancels)."""
    from oracle.metrics import memory_usage
    X = synth.power_law_tensor((300, 400, 30), 20000, 9, zipf_a=1.2)
    o = ora.ctd_s(X.dims, X.idx, X.val, 0, 300, 4, want_C=True)
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 300, 4)
        assert np.array_equal(h.result()["accepted"], o.accepted.astype(np.uint64))
        m = h.memory_usage()
    finally:
        h.close()
    nc, nu, nr, usage = memory_usage(o.R, o.C, X.nnz)
    assert (m["nnz_C"], m["nnz_U"], m["nnz_R"], m["nnz_X"]) == (nc, nu, nr, X.nnz)
    assert m["usage"] == pytest.approx(usage, rel=1e-15)


def test_memory_usage_ctd_d(lib):
    """Eq. 15 after CTD-D updates: nnz(X) counts every slice, and the counts
    equal the oracle's on the same stream (the cross-term rows of C fill in)."""
    from oracle.metrics import memory_usage
    st = synth.traffic_stream(dims=(60, 50, 12), nnz0=2500, n_slices=6, slice_nnz=(60, 400),
                              zipf_a=1.1, n_anomalies=1, block=6, seed=5)
    o = ora.Dynamic(st.initial.dims, st.initial.idx, st.initial.val, 0, 40, 5)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 40, 5)
        for sl in st.slices:
            o.update(sl.dims, sl.idx, sl.val, 6)
            sd, si, sv = lib.to_device(sl, "cuda")
            h.update(sd, si, sv, 6)
        assert np.array_equal(h.result()["accepted"], np.asarray(o.accepted, dtype=np.uint64))
        m = h.memory_usage()
    finally:
        h.close()
    total = st.initial.nnz + sum(sl.nnz for sl in st.slices)
    nc, nu, nr, usage = memory_usage(o.R, o.C, total)
    assert (m["nnz_U"], m["nnz_R"], m["nnz_X"]) == (nu, nr, total)
    assert m["nnz_C"] == nc


@pytest.mark.parametrize("which,precision", [("power", "fp64"), ("haggle", "mixed")])
def test_sparse_core_matches_oracle(lib, which, precision):
    """C_(alpha) = R^T X_(alpha) in compressed-column form (ctd_sparse_core)
    against the oracle's sparse product from its own R: same column pointers
    and row indices (positive values, so no entry cancels), values to
    rounding, and as many entries as Eq. 15 counts in the dense C."""
    import ctypes
    import torch
    from oracle.metrics import sparse_core
    if which == "power":
        X, s = synth.power_law_tensor((300, 400, 30), 20000, 9, zipf_a=1.2), 300
    else:
        X, s = synth.small_shapes()[1], 400
    o = ora.ctd_s(X.dims, X.idx, X.val, 0, s, 4)
    indptr, indices, data = sparse_core(o.R, ora.unfold(X.dims, X.idx, X.val, 0))
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision=precision, want_C=True)
    try:
        h.decompose(dims, idx, val, 0, s, 4)
        assert np.array_equal(h.result()["accepted"], o.accepted.astype(np.uint64))
        col_ptr, row_idx, vals = h.sparse_core()
        m = h.memory_usage()
        # too small a cap: the count comes back with CTD_ERR_CAPACITY, nothing else written
        cp = torch.empty(col_ptr.shape[0], dtype=torch.int64, device="cuda")
        nnz = ctypes.c_int64(-1)
        rc = h.lib.ctd_sparse_core(h.h, cp.data_ptr(), None, None, 0, ctypes.byref(nnz))
        assert rc == lib.CTD_ERR_CAPACITY and nnz.value == len(row_idx)
        assert np.array_equal(cp.cpu().numpy(), col_ptr)
    finally:
        h.close()
    assert np.array_equal(col_ptr, indptr)
    assert np.array_equal(row_idx, indices)
    np.testing.assert_allclose(vals, data, rtol=1e-13, atol=0)
    assert m["nnz_C"] == len(row_idx)


def test_sparse_core_needs_a_static_decomposition(lib):
    """After a CTD-D update the held C is a projection, not R^T X: state error."""
    st = synth.traffic_stream(dims=(40, 30, 8), nnz0=800, n_slices=1, slice_nnz=(50, 100),
                              zipf_a=1.1, n_anomalies=0, block=4, seed=2)
    dims, idx, val = lib.to_device(st.initial, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 30, 1)
        h.sparse_core()
        sd, si, sv = lib.to_device(st.slices[0], "cuda")
        h.update(sd, si, sv, 4)
        with pytest.raises(lib.CtdError):
            h.sparse_core()
    finally:
        h.close()

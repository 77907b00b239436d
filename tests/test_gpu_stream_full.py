"""CTD-D at full size: the 4,000 x 4,000 x 200 traffic stream (1M nonzeros, then
200 slices of 2k-50k nonzeros, dense bursts in slices 5, 81 and 196), s = 800,
d = 8, against stored oracle results (tests/golden/make_stream_4000.py, CPU
oracle only), one slice per call and in batches of 8, in both precisions.

Checked at the end of every call: the draws of its last slice and the kept
fibers bit for bit, the error of the grown decomposition (1e-6 relative in
float64, 1e-4 in mixed mode) and the norm.  At the end of the stream: 112
columns of C_(alpha) (64 seeded over the stream, 16 from each burst slice)
against their closed form R^T P_tau x (Eqs. 8-13 unrolled).
"""
import os

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "stream_4000_s800_d8.npz")
U64 = 2.0 ** -52


def _split(flat, lens):
    out, o = [], 0
    for n in lens:
        out.append(flat[o:o + n])
        o += n
    return out


@pytest.fixture(scope="module")
def stream():
    return synth.traffic_stream()


def core_tolerance(precision, cond_R):
    """Relative bound on C against its closed form (largest entry as the scale).

    float64: the library forms the cross rows as (M w)^T C with Q = R M
    orthonormal, so each row carries about u * cond(R) relative error per pass
    (|M w| <= |w| / sigma_min(R)); the bound allows 64 u cond(R).
    mixed: C is held in float32, the same with u32 = 2^-23 (64 u32 cond(R)
    would exceed 1, so float32 rounding of C and of the new rows, 2^-23 per
    entry relative to the column's scale, is bounded by 4096 u32)."""
    if precision == "fp64":
        return 64 * U64 * cond_R
    return 4096 * 2.0 ** -23


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,batch", [("fp64", 1), ("mixed", 1), ("fp64", 8), ("mixed", 8)])
def test_stream_full_size(stream, precision, batch):
    import paper_1710_03608_amd as ctd
    ctd.load_library()
    g = np.load(GOLD, allow_pickle=False)
    st = stream
    X = st.initial
    dims, idx, val = ctd.to_device(X, "cuda")
    h = ctd.Ctd(precision=precision, want_C=True)
    try:
        h.decompose(dims, idx, val, 0, 800, 0)
        r = h.result()
        assert np.array_equal(r["draws"], g["init_draws"])
        assert np.array_equal(r["unique"], g["init_unique"])
        assert np.array_equal(r["accepted"], g["init_accepted"])
        tol = 1e-6 if precision == "fp64" else 1e-4
        rel0 = float(g["init_err2"] / g["init_norm2"])
        assert abs(r["rel_err"] - rel0) <= tol * rel0 + 1e-12
        n = int(g["n_slices"])
        assert n == len(st.slices) == 200
        draws = _split(g["draws"], g["draws_len"])
        acc = _split(g["accepted"], g["accepted_len"])
        T0, J = X.dims[2], X.dims[1]
        held = list(g["init_accepted"])
        slices = [ctd.to_device(sl, "cuda") for sl in st.slices]
        for t in range(n):
            if batch == 1:
                h.update(*slices[t], 8)
            elif t % batch == 0:
                h.update_batched(slices[t:t + batch], 8)
            held.extend(acc[t].tolist())
            if (t + 1) % batch and t + 1 < n:
                continue
            r = h.result()
            off = np.uint64((T0 + t) * J)
            assert np.array_equal(r["draws"] + off, draws[t]), t      # draws of the last slice
            assert r["step"] == t + 1
            assert r["s_tilde"] == int(g["d_tilde"][t]), t
            assert r["n_cols"] == int(g["n_cols"][t]), t
            assert np.array_equal(r["accepted"], np.array(held, dtype=np.uint64)), t
            rel = float(g["err2"][t] / g["norm2"][t])
            assert abs(r["rel_err"] - rel) <= tol * rel + 1e-12, (t, r["rel_err"], rel)
            assert r["norm2"] == pytest.approx(float(g["norm2"][t]), rel=1e-12)
        full = h.result(factors=True, core=False)
        assert np.array_equal(full["accepted"], g["all_accepted"])
        assert np.array_equal(full["col_ids"][g["C_cols"]], g["C_fids"])
        Cg = h.core_columns(g["C_cols"]).astype(np.float64)
        ref = g["C_sample"]
        cond = np.linalg.cond(full["R"])
        err = np.abs(Cg - ref).max() / np.abs(ref).max()
        print(f"C vs closed form: {err:.3e} relative, cond(R) {cond:.3e}, "
              f"bound {core_tolerance(precision, cond):.3e}", flush=True)
        assert err <= core_tolerance(precision, cond), (err, cond)
    finally:
        h.close()

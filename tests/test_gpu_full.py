"""CTD-S at the benchmark's full size (5M nonzeros) against stored oracle results.

The expected values come from tests/golden/make_traffic_5m.py, which calls
only the CPU oracle.  Checked: draws, unique fibers, multiplicities and kept
fibers bit for bit; the relative error to 1e-6 (float64) or 1e-4 (mixed);
per-fiber residuals on a seeded sample of 4000 fibers.
"""
import os

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "traffic_5m_s2000_seed0.npz")


@pytest.fixture(scope="module")
def case():
    import torch
    import paper_1710_03608_amd as ctd
    ctd.load_library()
    X = synth.traffic_5m()
    g = np.load(GOLD, allow_pickle=False)
    dims, idx, val = ctd.to_device(X, "cuda")
    # squared norms of the sampled fibers, from the input itself
    f = X.idx[1].astype(np.int64) + X.idx[2].astype(np.int64) * X.dims[1]
    want = g["sample_fid"].astype(np.int64)
    pos = np.searchsorted(want, f)
    pos = np.minimum(pos, want.shape[0] - 1)
    hit = want[pos] == f
    norm2 = np.zeros(want.shape[0])
    np.add.at(norm2, pos[hit], X.val[hit] ** 2)
    return ctd, dims, idx, val, g, norm2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_parity(case, precision):
    ctd, dims, idx, val, g, norm2 = case
    h = ctd.Ctd(precision=precision, want_fiber_stats=True)
    try:
        h.decompose(dims, idx, val, 0, 2000, 0)
        r = h.result()
    finally:
        h.close()
    assert np.array_equal(r["draws"], g["draws"])
    assert np.array_equal(r["unique"], g["unique"])
    assert np.array_equal(r["counts"], g["counts"])
    assert np.array_equal(r["accepted"], g["accepted"])
    assert r["n_f"] == int(g["n_f"])
    rel_o = float(g["rel_err"])
    tol = 1e-6 if precision == "fp64" else 1e-4
    assert abs(r["rel_err"] - rel_o) <= tol * rel_o + 1e-12, (r["rel_err"], rel_o)
    pos = g["sample_pos"]
    assert np.array_equal(r["fiber_ids"][pos], g["sample_fid"])
    d = np.abs(r["fiber_resid"][pos] - g["sample_resid"])
    ftol = 1e-7 if precision == "fp64" else 1e-4
    assert np.all(d <= ftol * norm2 + 1e-12), float(np.max(d / np.maximum(norm2, 1e-300)))

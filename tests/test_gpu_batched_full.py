"""Batched CTD-S at full size: the 512 independent tensors of uneven shape (I, J
in 500..5000, K in 20..200, 10k-200k nonzeros, Zipf(1.2) degrees, uniform(0,1]
values), s_b = 5% of tensor b's non-empty fibers, one batched call in each
precision, against stored oracle results for 16 of the tensors whose sizes
span the range (tests/golden/make_many_512.py, CPU oracle only; tensor b
draws with Philox counter word b).

Checked per stored tensor: draws, unique fibers, multiplicities and kept
fibers bit for bit, and the error (1e-6 relative in float64, 1e-4 in mixed
mode); for every tensor of the call, the sizes and a finite error in [0, 1];
and the same call three times more (captured as a graph, then replayed), the
stored tensors' results bit for bit equal to the first call's.
"""
import math
import os

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "many_512_subset.npz")


def _split(flat, lens):
    out, o = [], 0
    for n in lens:
        out.append(flat[o:o + n])
        o += n
    return out


@pytest.fixture(scope="module")
def many():
    ts = synth.many_tensors()
    s = [max(1, math.ceil(0.05 * synth.count_nonempty_fibers(t, 0))) for t in ts]
    return ts, s


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_many_tensors_full_size(many, precision):
    import paper_1710_03608_amd as ctd
    ctd.load_library()
    g = np.load(GOLD, allow_pickle=False)
    ts, s = many
    assert len(ts) == 512
    sel = g["tensors"]
    assert [s[b] for b in sel] == g["s"].tolist()
    draws = _split(g["draws"], g["draws_len"])
    uniq = _split(g["unique"], g["unique_len"])
    counts = _split(g["counts"], g["counts_len"])
    acc = _split(g["accepted"], g["accepted_len"])
    rtol, atol = (1e-6, 1e-12) if precision == "fp64" else (1e-4, 1e-8)
    h = ctd.Ctd(precision=precision)
    try:
        devs = [ctd.to_device(t, "cuda") for t in ts]
        h.decompose_batched(devs, 0, s, 0)
        h.sync()
        for i, b in enumerate(sel.tolist()):
            r = h.batch_result(b)
            assert r["s"] == s[b]
            assert np.array_equal(r["draws"], draws[i]), b
            assert np.array_equal(r["unique"], uniq[i]), b
            assert np.array_equal(r["counts"], counts[i]), b
            assert np.array_equal(r["accepted"], acc[i]), b
            rel = float(g["err2"][i] / g["norm2"][i])
            assert abs(r["rel_err"] - rel) <= rtol * rel + atol, (b, r["rel_err"], rel)
        for b, t in enumerate(ts):
            r = h.batch_result(b, arrays=False)
            assert r["s"] == s[b] and 1 <= r["s_tilde"] <= min(r["s_unique"], t.dims[0]), b
            # a tensor whose kept fibers span all its rows has error 0 up to rounding
            assert -atol <= r["rel_err"] <= 1.0, (b, r["rel_err"])
        # the same call again is captured as a graph, then replayed: same bits
        first = [h.batch_result(b) for b in sel.tolist()]
        for rep in range(3):
            h.decompose_batched(devs, 0, s, 0)
            h.sync()
            assert h.batch_graph_launches() == rep + 1, rep   # capture, then replays
            for i, b in enumerate(sel.tolist()):
                r = h.batch_result(b)
                for key in ("draws", "unique", "counts", "accepted", "prob", "scale"):
                    assert np.array_equal(r[key], first[i][key]), (rep, b, key)
                assert r["err2"] == first[i]["err2"] and r["norm2"] == first[i]["norm2"], (rep, b)
    finally:
        h.close()

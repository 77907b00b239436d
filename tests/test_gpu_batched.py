"""Batched CTD-S (many independent tensors in one call) against the CPU oracle:
tensor b draws with Philox counter word tensor = b (oracle ctd_s(..., tensor=b))."""
import math

import numpy as np
import pytest

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


def _tensors(n, seed):
    """Uneven shapes and sizes shaped like the many-tensor workload, scaled down."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    for b in range(n):
        I, J, K = (int(rng.integers(30, 200)), int(rng.integers(30, 200)), int(rng.integers(4, 20)))
        nnz = int(rng.integers(300, 6000))
        out.append(synth.power_law_tensor((I, J, K), min(nnz, I * J * K // 4), 1000 + b, zipf_a=1.2,
                                          values="uniform"))
    return out


def _sizes(ts):
    return [max(1, math.ceil(0.05 * synth.count_nonempty_fibers(t, 0))) for t in ts]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_matches_oracle_per_tensor(lib, precision):
    ts = _tensors(19, 3)          # more tensors than internal streams
    s = _sizes(ts)
    h = lib.Ctd(precision=precision)
    try:
        h.decompose_batched([lib.to_device(t, "cuda") for t in ts], 0, s, 11)
        for b, t in enumerate(ts):
            o = ora.ctd_s(t.dims, t.idx, t.val, 0, s[b], 11, tensor=b)
            g = h.batch_result(b)
            assert np.array_equal(g["draws"], o.draws.astype(np.uint64)), b
            assert np.array_equal(g["unique"], o.uniq.astype(np.uint64)), b
            assert np.array_equal(g["counts"], o.counts.astype(np.int32)), b
            assert np.array_equal(g["accepted"], o.accepted.astype(np.uint64)), b
            assert np.allclose(g["scale"], o.omega, rtol=1e-13, atol=0)
            rtol, atol = (1e-6, 1e-12) if precision == "fp64" else (1e-4, 1e-8)
            assert abs(g["rel_err"] - o.rel_err) <= rtol * o.rel_err + atol, (b, g["rel_err"], o.rel_err)
    finally:
        h.close()


def test_tensor_zero_equals_single_and_state_is_kept(lib):
    ts = _tensors(3, 5)
    s = _sizes(ts)
    h = lib.Ctd()
    try:
        dims, idx, val = lib.to_device(ts[0], "cuda")
        h.decompose(dims, idx, val, 0, s[0], 2)
        single = h.result()
        h.decompose_batched([lib.to_device(t, "cuda") for t in ts], 0, s, 2)
        g0 = h.batch_result(0)
        assert np.array_equal(g0["draws"], single["draws"])
        assert np.array_equal(g0["accepted"], single["accepted"])
        # reductions split by how many tensors share a launch: equal to rounding
        assert g0["err2"] == pytest.approx(single["err2"], rel=1e-12)
        again = h.result()                      # the handle's own CTD-S result is untouched
        assert np.array_equal(again["accepted"], single["accepted"]) and again["err2"] == single["err2"]
        # a second batched call with other sizes reuses the handle
        h.decompose_batched([lib.to_device(t, "cuda") for t in ts[1:]], 0, s[1:], 2)
        g = h.batch_result(1)
        o = ora.ctd_s(ts[2].dims, ts[2].idx, ts[2].val, 0, s[2], 2, tensor=1)
        assert np.array_equal(g["accepted"], o.accepted.astype(np.uint64))
    finally:
        h.close()


def test_batched_argument_checks(lib):
    ts = _tensors(2, 7)
    h = lib.Ctd()
    try:
        dev = [lib.to_device(t, "cuda") for t in ts]
        with pytest.raises(lib.CtdError) as ei:
            h.decompose_batched(dev, 3, [5, 5], 0)
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
        with pytest.raises(lib.CtdError) as ei:
            h.decompose_batched(dev, 0, [5, 0], 0)
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
        with pytest.raises(lib.CtdError) as ei:
            h.batch_result(0)
        assert ei.value.name == "CTD_ERR_STATE"
        h.decompose_batched(dev, 0, [5, 5], 0)
        with pytest.raises(lib.CtdError) as ei:
            h.batch_result(2)
        assert ei.value.name == "CTD_ERR_INVALID_ARG"
        assert h.batch_result(1)["s"] == 5
    finally:
        h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_few_tensors_with_many_blocks(lib, precision):
    """Three tensors of several 64-candidate blocks each and uneven candidate
    counts: a launch this small uses the side-stream lookahead, and inputs
    drop out of later block steps as their candidates run out."""
    ts = [synth.power_law_tensor((120, 150, 12), 6000, 41, zipf_a=1.2, values="uniform"),
          synth.power_law_tensor((90, 200, 10), 5000, 42, zipf_a=1.2, values="uniform"),
          synth.power_law_tensor((200, 80, 15), 7000, 43, zipf_a=1.2, values="uniform")]
    s = [260, 150, 330]
    h = lib.Ctd(precision=precision)
    try:
        h.decompose_batched([lib.to_device(t, "cuda") for t in ts], 0, s, 6)
        for b, t in enumerate(ts):
            o = ora.ctd_s(t.dims, t.idx, t.val, 0, s[b], 6, tensor=b)
            g = h.batch_result(b)
            assert len(o.uniq) > 64, b      # at least two block steps
            assert np.array_equal(g["unique"], o.uniq.astype(np.uint64)), b
            assert np.array_equal(g["accepted"], o.accepted.astype(np.uint64)), b
            rtol, atol = (1e-6, 1e-12) if precision == "fp64" else (1e-4, 1e-8)
            assert abs(g["rel_err"] - o.rel_err) <= rtol * o.rel_err + atol, (b, g["rel_err"], o.rel_err)
    finally:
        h.close()


def test_large_tensor_in_a_batch_takes_the_hot_row_projection(lib):
    """A tensor of more than 2^18 nonzeros among small ones: its projection
    runs the hot-row split inside the batched call, also when the call is
    captured as a graph and replayed."""
    ts = [synth.power_law_tensor((1500, 500, 40), 300000, 45, zipf_a=1.3),
          synth.power_law_tensor((90, 200, 10), 5000, 42, zipf_a=1.2, values="uniform"),
          synth.power_law_tensor((200, 80, 15), 7000, 43, zipf_a=1.2, values="uniform")]
    s = [900, 60, 90]
    devs = [lib.to_device(t, "cuda") for t in ts]
    h = lib.Ctd()
    try:
        h.decompose_batched(devs, 0, s, 7)
        ref = _batch_snapshot(h, len(ts))
        for b, t in enumerate(ts):
            o = ora.ctd_s(t.dims, t.idx, t.val, 0, s[b], 7, tensor=b)
            g = h.batch_result(b)
            assert np.array_equal(g["accepted"], o.accepted.astype(np.uint64)), b
            assert abs(g["rel_err"] - o.rel_err) <= 1e-6 * o.rel_err + 1e-12, (b, g["rel_err"], o.rel_err)
        for rep in range(3):                      # captured, then replayed twice
            h.decompose_batched(devs, 0, s, 7)
            _same(_batch_snapshot(h, len(ts)), ref)
        assert h.batch_graph_launches() == 3
    finally:
        h.close()


def _batch_snapshot(h, n):
    out = []
    for b in range(n):
        r = h.batch_result(b)
        out.append((r["draws"].copy(), r["unique"].copy(), r["counts"].copy(), r["accepted"].copy(),
                    r["scale"].copy(), r["prob"].copy(), r["err2"], r["norm2"], r["s_tilde"], r["s_unique"]))
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            if isinstance(u, np.ndarray):
                assert u.dtype == v.dtype and np.array_equal(u.view(np.uint8), v.view(np.uint8))
            else:
                assert u == v


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_repeated_calls_replay_a_graph_bit_identically(lib, precision):
    """A batched call repeated with the same inputs and sizes is captured once
    (second call) and replayed after that: every replay, with eager work and
    synchronizations of the program between them, gives the eager call's bits;
    a call with other sizes runs directly, and a replay reads the current
    values of the (same) input buffers.  The handles run on torch's default
    stream, which cannot be captured itself: the graph runs on a stream of the
    handle forked from it, and the launch count shows that it did."""
    import torch
    ts = _tensors(19, 7)
    s = _sizes(ts)
    devs = [lib.to_device(t, "cuda") for t in ts]
    h = lib.Ctd(precision=precision)
    other = lib.Ctd(precision=precision)
    try:
        h.decompose_batched(devs, 0, s, 5)
        ref = _batch_snapshot(h, len(ts))
        assert h.batch_graph_launches() == 0
        for rep in range(5):                      # capture at rep 0, replays after it
            h.decompose_batched(devs, 0, s, 5)
            other.decompose(*devs[rep], 0, s[rep], 9)   # eager work in between
            other.result()
            torch.cuda.synchronize()
            _same(_batch_snapshot(h, len(ts)), ref)
            assert h.batch_graph_launches() == rep + 1
        s2 = list(s)
        s2[0] += 1                                # another signature: direct launches
        h.decompose_batched(devs, 0, s2, 5)
        o = ora.ctd_s(ts[0].dims, ts[0].idx, ts[0].val, 0, s2[0], 5, tensor=0)
        assert np.array_equal(h.batch_result(0)["accepted"], o.accepted.astype(np.uint64))
        assert h.batch_graph_launches() == 5
        for rep in range(3):                      # back: direct, capture, replay
            h.decompose_batched(devs, 0, s, 5)
            _same(_batch_snapshot(h, len(ts)), ref)
        assert h.batch_graph_launches() == 7
        # new values in the same buffers of tensor 3: the replay reads them
        rng = np.random.default_rng(4)
        newval = rng.uniform(0.5, 2.0, size=ts[3].val.shape)
        devs[3][2].copy_(torch.as_tensor(newval, dtype=devs[3][2].dtype, device="cuda"))
        h.decompose_batched(devs, 0, s, 5)
        assert h.batch_graph_launches() == 8
        got = h.batch_result(3)
        o = ora.ctd_s(ts[3].dims, ts[3].idx, newval, 0, s[3], 5, tensor=3)
        assert np.array_equal(got["draws"], o.draws.astype(np.uint64))
        assert np.array_equal(got["accepted"], o.accepted.astype(np.uint64))
        rtol, atol = (1e-6, 1e-12) if precision == "fp64" else (1e-4, 1e-8)
        assert abs(got["rel_err"] - o.rel_err) <= rtol * o.rel_err + atol
    finally:
        other.close()
        h.close()

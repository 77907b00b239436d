"""Allocation failures injected into the library (CTD_FAIL_ALLOC): every
device allocation of a call can fail as if the device were out of memory,
the call reports CTD_ERR_OOM with a message, and the handle then works
again and gives the results of a handle that never failed."""
import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1710_03608_amd as ctd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctd.load_library()
    return ctd


def _same(a, b):
    assert np.array_equal(a["draws"], b["draws"])
    assert np.array_equal(a["accepted"], b["accepted"])
    assert a["err2"] == b["err2"] and a["norm2"] == b["norm2"]


def test_failed_allocations_of_a_decomposition(lib, monkeypatch):
    X = synth.power_law_tensor((300, 200, 60), 40000, 4, zipf_a=1.2)
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd()
    try:
        h.decompose(dims, idx, val, 0, 300, 3)
        ref = h.result()
    finally:
        h.close()
    failed = []
    for k in range(1, 6):                 # the scalars, the workspace, the basis arguments, ...
        monkeypatch.setenv("CTD_FAIL_ALLOC", str(k))
        h = None
        try:
            h = lib.Ctd()
            h.decompose(dims, idx, val, 0, 300, 3)
            got = h.result()
            _same(got, ref)                # the k-th allocation lies beyond this call
        except lib.CtdError as e:
            assert e.name == "CTD_ERR_OOM", str(e)
            assert "alloc" in str(e).lower(), str(e)
            failed.append(k)
        monkeypatch.delenv("CTD_FAIL_ALLOC")
        if h is not None:
            try:
                h.decompose(dims, idx, val, 0, 300, 3)
                _same(h.result(), ref)
            finally:
                h.close()
    assert failed[:3] == [1, 2, 3], failed


def test_failed_allocations_of_a_batched_call(lib, monkeypatch):
    ts = [synth.power_law_tensor((120, 150, 12), 6000, 41, zipf_a=1.2, values="uniform"),
          synth.power_law_tensor((90, 200, 10), 5000, 42, zipf_a=1.2, values="uniform"),
          synth.power_law_tensor((200, 80, 15), 7000, 43, zipf_a=1.2, values="uniform")]
    s = [80, 60, 90]
    devs = [lib.to_device(t, "cuda") for t in ts]
    h = lib.Ctd()
    try:
        h.decompose_batched(devs, 0, s, 6)
        ref = [h.batch_result(b) for b in range(3)]
    finally:
        h.close()
    h = lib.Ctd()
    failed = 0
    try:
        for k in range(1, 30):
            monkeypatch.setenv("CTD_FAIL_ALLOC", str(k))
            try:
                h.decompose_batched(devs, 0, s, 6)
                h.sync()
            except lib.CtdError as e:
                assert e.name == "CTD_ERR_OOM", str(e)
                failed += 1
            monkeypatch.delenv("CTD_FAIL_ALLOC")
            h.decompose_batched(devs, 0, s, 6)
            for b in range(3):
                _same(h.batch_result(b), ref[b])
    finally:
        h.close()
    assert failed >= 1

"""ctd_sparse_core_noalloc (the variant for callers that cannot allocate: its
workspace lives in the library's static per-GPU scratch) against
ctd_sparse_core, through the C ABI: two decompositions in a row, the second
on a smaller input, each compared bit for bit (same kernels, same order of
additions), and a repeat of the first after the second (the scratch keeps the
last call's contents, which must not leak into a result)."""
import ctypes

import numpy as np
import pytest

from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1710_03608_amd as ctd
    assert torch.cuda.is_available()
    ctd.load_library()
    return ctd


def _pair(lib, X, s, seed):
    dims, idx, val = lib.to_device(X, "cuda")
    h = lib.Ctd(precision="fp64", want_C=True)
    try:
        h.decompose(dims, idx, val, 0, s, seed)
        ref = h.sparse_core()
        got = h.sparse_core(noalloc=True)
        # the capacity protocol of the variant: count only, CTD_ERR_CAPACITY
        import torch
        cp = torch.empty(ref[0].shape[0], dtype=torch.int64, device="cuda")
        nnz = ctypes.c_int64(-1)
        rc = h.lib.ctd_sparse_core_noalloc(h.h, cp.data_ptr(), None, None, 0, ctypes.byref(nnz))
        if len(ref[1]):
            assert rc == lib.CTD_ERR_CAPACITY
        assert nnz.value == len(ref[1])
        assert np.array_equal(cp.cpu().numpy(), ref[0])
    finally:
        h.close()
    return ref, got


def _same(ref, got):
    for a, b in zip(ref, got):
        assert a.dtype == b.dtype and a.shape == b.shape
        assert np.array_equal(a, b)


def test_noalloc_matches_sparse_core_on_two_calls(lib):
    big = synth.power_law_tensor((2000, 1500, 40), 200_000, 21, zipf_a=1.2)
    small = synth.power_law_tensor((300, 400, 30), 20_000, 9, zipf_a=1.2)
    ref1, got1 = _pair(lib, big, 600, 3)
    assert len(ref1[1]) > 100_000
    _same(ref1, got1)
    ref2, got2 = _pair(lib, small, 300, 4)
    assert 0 < len(ref2[1]) < len(ref1[1])
    _same(ref2, got2)
    ref3, got3 = _pair(lib, big, 600, 3)
    _same(ref1, ref3)
    _same(ref1, got3)

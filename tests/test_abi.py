"""The C-ABI library loads and exports every entry point its header declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctd.h")
LIB = os.path.join(ROOT, "paper_1710_03608_amd", "libctd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    assert names == sorted(["ctd_create", "ctd_decompose", "ctd_decompose_given", "ctd_update",
                            "ctd_update_batched", "ctd_decompose_batched", "ctd_get_batch_result",
                            "ctd_sync", "ctd_get_result", "ctd_last_error", "ctd_destroy",
                            "ctd_attack_candidates", "ctd_memory_usage", "ctd_sparse_core"])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctd.so not built")
def test_binding_struct_layout_matches_exports():
    import paper_1710_03608_amd as ctd
    lib = ctd.load_library()
    for name in ctd.EXPORTS:
        assert hasattr(lib, name)
    # ctd_create rejects a NULL out pointer without touching the GPU
    assert lib.ctd_create(None, None, None) == 1
    assert lib.ctd_last_error(None) == b"null handle"
    assert lib.ctd_update_batched(None, None, 1, 1) == 1
    assert lib.ctd_decompose_batched(None, None, 1, 0, None, 0) == 1
    assert lib.ctd_get_batch_result(None, 0, None) == 1
    assert lib.ctd_attack_candidates(None, 1, None, None, 0, None, None) == 1
    assert lib.ctd_memory_usage(None, None) == 1
    assert lib.ctd_sparse_core(None, None, None, None, 0, None) == 1

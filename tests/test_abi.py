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
                            "ctd_attack_candidates", "ctd_memory_usage", "ctd_sparse_core",
                            "ctd_sparse_core_noalloc", "ctd_save_state", "ctd_load_state",
                            "ctd_batch_graph_launches"])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctd.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (its HIP runtime is the one the library binds to)
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
    assert lib.ctd_sparse_core_noalloc(None, None, None, None, 0, None) == 1
    assert lib.ctd_save_state(None, None, None) == 1
    assert lib.ctd_load_state(None, None, 0) == 1


SANITIZED = os.path.join(ROOT, "paper_1710_03608_amd", "libctd_asan.so")
SANITIZED_CHECKS = r"""
import ctypes, sys
lib = ctypes.CDLL(sys.argv[1])
lib.ctd_last_error.restype = ctypes.c_char_p
lib.ctd_last_error.argtypes = [ctypes.c_void_p]
class Opt(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("eps", ctypes.c_double), ("want_C", ctypes.c_int32),
                ("want_fiber_stats", ctypes.c_int32), ("profile", ctypes.c_int32)]
h = ctypes.c_void_p()
assert lib.ctd_create(None, None, None) == 1
assert lib.ctd_last_error(None) == b"null handle"
for bad in (Opt(5, 1e-6, 0, 0, 0), Opt(0, -1.0, 0, 0, 0), Opt(0, 1.0, 0, 0, 0)):
    assert lib.ctd_create(ctypes.byref(h), ctypes.byref(bad), None) == 1 and not h.value
rc = lib.ctd_create(ctypes.byref(h), None, None)       # no GPU here: the runtime error path
assert rc in (0, 6 , 7), rc
if rc == 0:
    lib.ctd_destroy(h)
else:
    assert b"hipMalloc" in lib.ctd_last_error(None)
for name, args in (("ctd_decompose", (None, None, 0, 1, 0)), ("ctd_update", (None, None, 1)),
                   ("ctd_update_batched", (None, None, 1, 1)), ("ctd_sync", (None,)),
                   ("ctd_get_result", (None, None)), ("ctd_memory_usage", (None, None)),
                   ("ctd_sparse_core", (None, None, None, None, 0, None)),
                   ("ctd_sparse_core_noalloc", (None, None, None, None, 0, None)),
                   ("ctd_save_state", (None, None, None)), ("ctd_load_state", (None, None, 0)),
                   ("ctd_decompose_batched", (None, None, 1, 0, None, 0)),
                   ("ctd_get_batch_result", (None, 0, None)),
                   ("ctd_attack_candidates", (None, 1, None, None, 0, None, None))):
    assert getattr(lib, name)(*args) == 1, name
lib.ctd_destroy(None)
print("sanitized host checks ok")
"""


@pytest.mark.skipif(not os.path.exists(SANITIZED), reason="libctd_asan.so not built")
def test_sanitized_library_host_paths():
    """The host code built with AddressSanitizer and UndefinedBehaviorSanitizer
    (paper_1710_03608_amd/build_asan.py) runs the argument checks, the option
    validation and the failed-create path without a report."""
    import glob
    import subprocess
    import sys
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang's ASan runtime is not installed")
    env = dict(os.environ, LD_PRELOAD=rts[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", SANITIZED_CHECKS, SANITIZED], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized host checks ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr

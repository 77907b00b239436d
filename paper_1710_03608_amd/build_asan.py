"""Build libctd_asan.so: the library with its host code under AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged), for the CPU-side tests of the
host logic.  Loaded into a process that preloads clang's ASan runtime
(ASAN_RUNTIME below); never used on a GPU."""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build_asan")
LIB = os.path.join(HERE, "libctd_asan.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-function", "-Wno-unknown-pragmas"] + HOST_SAN


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    r = subprocess.run([HIPCC, *FLAGS, "-c", os.path.join(SRC, src), "-o", obj],
                       capture_output=True, text=True)
    return src, obj, r


def build():
    from build_lib import SOURCES
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        for src, obj, r in ex.map(_compile, SOURCES):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc (sanitized host) failed on {src}")
            objs.append(obj)
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-shared-libsan",
                        "-o", tmp, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libctd_asan.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    sys.path.insert(0, HERE)
    print(build())

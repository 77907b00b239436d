"""Python binding of the MI355X CTD library (libctd.so, C ABI in include/ctd.h).

Argument marshalling only: every step of CTD-S / CTD-D runs in the HIP
kernels of libctd.so.  PyTorch supplies device memory and the stream.  The
binding fails loudly when the library has not been built; there is no CPU
path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctd.so")

CTD_F64, CTD_F32 = 0, 1
CTD_PREC_FP64, CTD_PREC_MIXED = 0, 1
STATUS = {0: "CTD_OK", 1: "CTD_ERR_INVALID_ARG", 2: "CTD_ERR_EMPTY", 3: "CTD_ERR_INDEX_OOB",
          4: "CTD_ERR_DUPLICATE", 5: "CTD_ERR_NONFINITE", 6: "CTD_ERR_OOM", 7: "CTD_ERR_HIP",
          8: "CTD_ERR_STATE", 9: "CTD_ERR_CAPACITY"}
CTD_ERR_CAPACITY = 9
EXPORTS = ("ctd_create", "ctd_decompose", "ctd_decompose_given", "ctd_update",
           "ctd_update_batched", "ctd_decompose_batched", "ctd_get_batch_result", "ctd_sync",
           "ctd_get_result", "ctd_last_error", "ctd_destroy", "ctd_attack_candidates",
           "ctd_memory_usage", "ctd_sparse_core", "ctd_sparse_core_noalloc", "ctd_save_state",
           "ctd_load_state", "ctd_batch_graph_launches")

c_i32, c_i64, c_u64, c_dbl, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_void_p)


class CooStruct(ctypes.Structure):
    _fields_ = [("order", c_i32), ("dims", ctypes.POINTER(c_i64)), ("nnz", c_i64),
                ("idx", c_vp), ("val", c_vp), ("val_dtype", c_i32)]


class OptionsStruct(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("eps", c_dbl), ("want_C", c_i32),
                ("want_fiber_stats", c_i32), ("profile", c_i32)]


class ResultStruct(ctypes.Structure):
    _fields_ = [("s", c_i64), ("s_unique", c_i64), ("s_tilde", c_i64), ("n_f", c_i64),
                ("n_rows", c_i64), ("step", c_i64), ("weight_total", c_u64),
                ("norm2", c_dbl), ("err2", c_dbl), ("rel_err", c_dbl), ("slice_err2", c_dbl),
                ("status", c_i32), ("stage_ms", ctypes.c_float * 8),
                ("draws", c_vp), ("unique", c_vp), ("counts", c_vp), ("prob", c_vp),
                ("scale", c_vp), ("accepted", c_vp),
                ("Q", c_vp), ("ldq", c_i64), ("Linv_t", c_vp), ("ldx", c_i64),
                ("R", c_vp), ("ldr", c_i64), ("C", c_vp), ("ldc", c_i64), ("n_cols", c_i64),
                ("col_ids", c_vp), ("fiber_ids", c_vp), ("fiber_resid", c_vp),
                ("C_dtype", c_i32)]


class MemoryStruct(ctypes.Structure):
    _fields_ = [("nnz_C", c_i64), ("nnz_U", c_i64), ("nnz_R", c_i64), ("nnz_X", c_i64),
                ("usage", ctypes.c_double)]


class CtdError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


_lib = None
_hip = None


def load_library():
    """Load libctd.so (built by build_lib.py); raise if it is missing.

    torch is imported first: its HIP runtime must be the one libctd.so binds
    to.  Loaded the other way round, the library's dependency would pull a
    second HIP (and HSA) runtime from the system into the process, and
    whichever initializes second finds no device."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python paper_1710_03608_amd/build_lib.py")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ctd_create.argtypes = [ctypes.POINTER(c_vp), ctypes.POINTER(OptionsStruct), c_vp]
    lib.ctd_decompose.argtypes = [c_vp, ctypes.POINTER(CooStruct), c_i32, c_i64, c_u64]
    lib.ctd_decompose_given.argtypes = [c_vp, ctypes.POINTER(CooStruct), c_i32,
                                        ctypes.POINTER(c_u64), c_i64]
    lib.ctd_update.argtypes = [c_vp, ctypes.POINTER(CooStruct), c_i64]
    lib.ctd_update_batched.argtypes = [c_vp, ctypes.POINTER(CooStruct), c_i32, c_i64]
    lib.ctd_decompose_batched.argtypes = [c_vp, ctypes.POINTER(CooStruct), c_i32, c_i32,
                                          ctypes.POINTER(c_i64), c_u64]
    lib.ctd_get_batch_result.argtypes = [c_vp, c_i32, ctypes.POINTER(ResultStruct)]
    lib.ctd_sync.argtypes = [c_vp]
    lib.ctd_get_result.argtypes = [c_vp, ctypes.POINTER(ResultStruct)]
    lib.ctd_last_error.argtypes = [c_vp]
    lib.ctd_last_error.restype = ctypes.c_char_p
    lib.ctd_destroy.argtypes = [c_vp]
    lib.ctd_destroy.restype = None
    lib.ctd_attack_candidates.argtypes = [c_vp, c_i32, c_vp, c_vp, c_i64,
                                          ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]
    lib.ctd_memory_usage.argtypes = [c_vp, ctypes.POINTER(MemoryStruct)]
    lib.ctd_sparse_core.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]
    lib.ctd_sparse_core_noalloc.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]
    lib.ctd_save_state.argtypes = [c_vp, c_vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.ctd_load_state.argtypes = [c_vp, c_vp, ctypes.c_size_t]
    lib.ctd_batch_graph_launches.argtypes = [c_vp]
    lib.ctd_batch_graph_launches.restype = c_i64
    for name in ("ctd_create", "ctd_decompose", "ctd_decompose_given", "ctd_update",
                 "ctd_update_batched", "ctd_decompose_batched", "ctd_get_batch_result",
                 "ctd_sync", "ctd_get_result", "ctd_attack_candidates", "ctd_memory_usage",
                 "ctd_sparse_core", "ctd_sparse_core_noalloc", "ctd_save_state", "ctd_load_state"):
        getattr(lib, name).restype = c_i32
    _lib = lib
    return lib


def _hip_runtime():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("HIP runtime library not found")
        _hip.hipMemcpy.argtypes = [c_vp, c_vp, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def device_to_numpy(ptr, count, dtype):
    """Copy `count` elements at device address `ptr` into a new numpy array."""
    dtype = np.dtype(dtype)
    out = np.empty(int(count), dtype=dtype)
    if count == 0 or not ptr:
        return out
    rc = _hip_runtime().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # DeviceToHost
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out


def device_columns(ptr, ld, rows, cols, dtype=np.float64):
    """Columns `cols` (first `rows` entries each) of a column-major device matrix."""
    dtype = np.dtype(dtype)
    out = np.empty((rows, len(cols)), dtype=dtype)
    for j, c in enumerate(cols):
        out[:, j] = device_to_numpy(ptr + int(c) * ld * dtype.itemsize, rows, dtype)
    return out


def device_matrix(ptr, rows, cols, ld, dtype=np.float64, row_major=True):
    flat = device_to_numpy(ptr, rows * ld if row_major else cols * ld, dtype)
    if row_major:
        return flat.reshape(rows, ld)[:, :cols].copy()
    return flat.reshape(cols, ld)[:, :rows].T.copy()


class Coo:
    """Keeps a COO tensor's device buffers alive and builds the C struct."""

    def __init__(self, dims, idx, val):
        import torch
        self.dims_arr = (c_i64 * len(dims))(*[int(d) for d in dims])
        self.idx = idx if idx.is_contiguous() else idx.contiguous()
        self.val = val if val.is_contiguous() else val.contiguous()
        assert self.idx.dtype == torch.int32 and self.idx.is_cuda
        assert self.val.is_cuda and self.val.dtype in (torch.float64, torch.float32)
        self.struct = CooStruct(len(dims), self.dims_arr, int(self.val.numel()),
                                self.idx.data_ptr() if self.val.numel() else None,
                                self.val.data_ptr() if self.val.numel() else None,
                                CTD_F64 if self.val.dtype == torch.float64 else CTD_F32)


def to_device(tensor_like, device="cuda", val_dtype="f64"):
    """numpy COO (dims, idx[N, nnz], val[nnz]) -> (dims, torch idx, torch val) on `device`."""
    import torch
    dims, idx, val = tensor_like.dims, tensor_like.idx, tensor_like.val
    ti = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32)).to(device)
    tv = torch.as_tensor(np.ascontiguousarray(val)).to(device)
    if val_dtype == "f32":
        tv = tv.float()
    return dims, ti, tv


class Ctd:
    """One handle of the CTD library bound to torch's current stream."""

    STAGES = ("sort", "sample", "panel", "basis", "project", "spmm", "core", "total")

    def __init__(self, precision="fp64", eps=1e-6, want_C=False, want_fiber_stats=False,
                 stream=None, profile=False):
        import torch
        lib = load_library()
        self.lib = lib
        opt = OptionsStruct(CTD_PREC_MIXED if precision == "mixed" else CTD_PREC_FP64,
                            float(eps), int(bool(want_C)), int(bool(want_fiber_stats)),
                            int(bool(profile)))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_vp()
        rc = lib.ctd_create(ctypes.byref(h), ctypes.byref(opt), c_vp(stream.cuda_stream))
        if rc != 0:
            raise CtdError(rc, "ctd_create: " + lib.ctd_last_error(None).decode())
        self.h = h
        self._keep = []

    def _check(self, rc):
        if rc != 0:
            raise CtdError(rc, self.lib.ctd_last_error(self.h).decode())

    def _hold(self, *objs):
        """Keep a call's input buffers alive until the stream has passed the call.

        Each call's buffers are held with an event recorded after it; holdings
        whose events have completed are released at the next call, so a long
        CTD-D stream does not accumulate its slices."""
        import torch
        self._keep = [(ev, o) for ev, o in self._keep if ev is not None and not ev.query()]
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self._keep.append((ev, objs))

    def decompose(self, dims, idx, val, mode, s, seed):
        coo = Coo(dims, idx, val)
        rc = self.lib.ctd_decompose(self.h, ctypes.byref(coo.struct), int(mode), int(s), int(seed))
        self._hold(coo)
        self._check(rc)

    def decompose_given(self, dims, idx, val, mode, draws):
        coo = Coo(dims, idx, val)
        arr = np.ascontiguousarray(np.asarray(draws, dtype=np.uint64))
        ptr = arr.ctypes.data_as(ctypes.POINTER(c_u64))
        rc = self.lib.ctd_decompose_given(self.h, ctypes.byref(coo.struct), int(mode), ptr,
                                          int(arr.shape[0]))
        self._hold(coo)
        self._check(rc)

    def update(self, dims, idx, val, d):
        coo = Coo(dims, idx, val)
        rc = self.lib.ctd_update(self.h, ctypes.byref(coo.struct), int(d))
        self._hold(coo)
        self._check(rc)

    def update_batched(self, slices, d):
        """CTD-D on consecutive slices [(dims, idx, val), ...] in one call."""
        coos = [Coo(dims, idx, val) for dims, idx, val in slices]
        arr = (CooStruct * len(coos))(*[c.struct for c in coos])
        rc = self.lib.ctd_update_batched(self.h, arr, len(coos), int(d))
        self._hold(coos, arr)
        self._check(rc)

    def decompose_batched(self, tensors, mode, s, seed):
        """CTD-S of many tensors [(dims, idx, val), ...] with s[b] draws each."""
        coos = [Coo(dims, idx, val) for dims, idx, val in tensors]
        arr = (CooStruct * len(coos))(*[c.struct for c in coos])
        sz = (c_i64 * len(coos))(*[int(x) for x in s])
        rc = self.lib.ctd_decompose_batched(self.h, arr, len(coos), int(mode), sz, int(seed))
        self._hold(coos, arr, sz)
        self._check(rc)

    def batch_graph_launches(self):
        """Batched calls of this handle that ran as a graph launch (capture or replay)."""
        return int(self.lib.ctd_batch_graph_launches(self.h))

    def batch_result(self, b, arrays=True):
        """Scalars (and index arrays) of tensor b of the last batched call."""
        r = ResultStruct()
        self._check(self.lib.ctd_get_batch_result(self.h, int(b), ctypes.byref(r)))
        out = {k: getattr(r, k) for k in ("s", "s_unique", "s_tilde", "n_f", "n_rows",
                                          "weight_total", "norm2", "err2", "rel_err")}
        if arrays:
            out["draws"] = device_to_numpy(r.draws, r.s, np.uint64)
            out["unique"] = device_to_numpy(r.unique, r.s_unique, np.uint64)
            out["counts"] = device_to_numpy(r.counts, r.s_unique, np.int32)
            out["prob"] = device_to_numpy(r.prob, r.s_unique, np.float64)
            out["scale"] = device_to_numpy(r.scale, r.s_unique, np.float64)
            out["accepted"] = device_to_numpy(r.accepted, r.s_tilde, np.uint64)
        return out

    def sync(self):
        self._check(self.lib.ctd_sync(self.h))

    def sparse_core(self, noalloc=False):
        """C_(alpha) = R^T X_(alpha) in compressed-column form (col_ptr, row_idx,
        vals as numpy arrays); device buffers sized from a first call with cap 0.
        noalloc=True calls ctd_sparse_core_noalloc (workspace in the library's
        static scratch) instead of ctd_sparse_core."""
        import torch
        fn = self.lib.ctd_sparse_core_noalloc if noalloc else self.lib.ctd_sparse_core
        n_f = self.result(arrays=False)["n_f"]
        col_ptr = torch.empty(n_f + 1, dtype=torch.int64, device="cuda")
        nnz = c_i64(0)
        rc = fn(self.h, col_ptr.data_ptr(), None, None, 0, ctypes.byref(nnz))
        if rc != CTD_ERR_CAPACITY or nnz.value == 0:
            self._check(rc)
        row_idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
        vals = torch.empty(max(nnz.value, 1), dtype=torch.float64, device="cuda")
        self._check(fn(self.h, col_ptr.data_ptr(), row_idx.data_ptr(), vals.data_ptr(), nnz.value,
                       ctypes.byref(nnz)))
        n = nnz.value
        return (col_ptr.cpu().numpy(), row_idx[:n].cpu().numpy(), vals[:n].cpu().numpy())

    def save_state(self):
        """Checkpoint of the CTD-D stream as a numpy uint8 array (host memory)."""
        n = ctypes.c_size_t(0)
        self._check(self.lib.ctd_save_state(self.h, None, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.ctd_save_state(self.h, buf.ctypes.data_as(c_vp), ctypes.byref(n)))
        return buf

    def load_state(self, buf):
        """Resume the CTD-D stream of a checkpoint made by save_state."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.ctd_load_state(self.h, buf.ctypes.data_as(c_vp), buf.nbytes))

    def memory_usage(self):
        """Eq. 15: nnz of C, U (structural) and R, nnz of the input, and the ratio."""
        m = MemoryStruct()
        self._check(self.lib.ctd_memory_usage(self.h, ctypes.byref(m)))
        return {"nnz_C": m.nnz_C, "nnz_U": m.nnz_U, "nnz_R": m.nnz_R, "nnz_X": m.nnz_X,
                "usage": m.usage}

    def attack_candidates(self, group_mode, cap=4096):
        """Candidates read off R: fiber ids and norms (host arrays), plus the
        number of groups (representatives)."""
        fids = np.zeros(max(cap, 1), dtype=np.uint64)
        norms = np.zeros(max(cap, 1), dtype=np.float64)
        n = c_i64(0)
        g = c_i64(0)
        self._check(self.lib.ctd_attack_candidates(
            self.h, int(group_mode), fids.ctypes.data_as(c_vp), norms.ctypes.data_as(c_vp),
            int(cap), ctypes.byref(n), ctypes.byref(g)))
        m = min(n.value, cap)
        return {"fids": fids[:m].copy(), "norms": norms[:m].copy(), "count": n.value,
                "n_groups": g.value}

    def raw_result(self):
        r = ResultStruct()
        self._check(self.lib.ctd_get_result(self.h, ctypes.byref(r)))
        return r

    def core_columns(self, cols):
        """Selected columns of C_(alpha) (s~ rows each), copied to the host."""
        r = self.raw_result()
        if not r.C:
            raise CtdError(8, "no C held")
        return device_columns(r.C, r.ldc, r.s_tilde, cols,
                              np.float32 if r.C_dtype == 1 else np.float64)

    def result(self, arrays=True, factors=False, core=True):
        """Scalars plus host copies of the index arrays (and factors if asked;
        core=False leaves out C itself, keeping its column ids)."""
        r = self.raw_result()
        out = {k: getattr(r, k) for k in ("s", "s_unique", "s_tilde", "n_f", "n_rows", "step",
                                          "weight_total", "norm2", "err2", "rel_err",
                                          "slice_err2", "n_cols")}
        out["stage_ms"] = dict(zip(self.STAGES, [float(x) for x in r.stage_ms]))
        if arrays:
            out["draws"] = device_to_numpy(r.draws, r.s, np.uint64)
            out["unique"] = device_to_numpy(r.unique, r.s_unique, np.uint64)
            out["counts"] = device_to_numpy(r.counts, r.s_unique, np.int32)
            out["prob"] = device_to_numpy(r.prob, r.s_unique, np.float64)
            out["scale"] = device_to_numpy(r.scale, r.s_unique, np.float64)
            out["accepted"] = device_to_numpy(r.accepted, r.s_tilde, np.uint64)
            if r.fiber_resid:
                out["fiber_ids"] = device_to_numpy(r.fiber_ids, r.n_f, np.uint64)
                out["fiber_resid"] = device_to_numpy(r.fiber_resid, r.n_f, np.float64)
        if factors:
            k = r.s_tilde
            out["Q"] = device_matrix(r.Q, r.n_rows, k, r.ldq)
            out["Linv_t"] = device_matrix(r.Linv_t, k, k, r.ldx)
            if r.R:
                out["R"] = device_matrix(r.R, r.n_rows, k, r.ldr)
            if r.C:
                if core:
                    out["C"] = device_matrix(r.C, k, r.n_cols, r.ldc, row_major=False,
                                             dtype=np.float32 if r.C_dtype == 1 else np.float64)
                out["col_ids"] = device_to_numpy(r.col_ids, r.n_cols, np.uint64)
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.ctd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Thin ctypes binding of libspmv.so (the C-ABI of ``include/spmv.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
Device vectors are torch tensors on ``cuda`` (ROCm); host arrays are numpy.
The library must be built (``__graft_entry__.build()``); importing this
module without it, or using it without a GPU, raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmv.so")

FMT = {"csr": 0, "csr5": 1, "ell": 2, "sell": 3, "hyb": 4}
FMT_NAMES = ("csr", "csr5", "ell", "sell", "hyb")
F64, F32 = 0, 1
NPARAM = 5317
NOALLOC_MAX_BATCH = 4096  # SPMV_NOALLOC_MAX_BATCH

STATUS = {0: "ok", -1: "invalid argument", -2: "bad structure", -3: "out of memory", -4: "too large",
          -5: "unsupported", -6: "HIP error", -7: "model error"}


class SpmvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("sell_C", ctypes.c_int32), ("sell_sigma", ctypes.c_int32), ("csr_lanes_per_row", ctypes.c_int32),
                ("hyb_K", ctypes.c_int32), ("csr5_omega", ctypes.c_int32), ("csr5_sigma", ctypes.c_int32),
                ("max_bytes", ctypes.c_int64), ("flags", ctypes.c_uint32), ("bands", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def params(**kw) -> Params:
    p = Params()
    p.hyb_K = -1
    for k, v in kw.items():
        setattr(p, k, int(v))
    return p


class Info(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("dtype", ctypes.c_int32), ("M", ctypes.c_int64), ("N", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("bytes_fmt", ctypes.c_int64), ("bytes_min", ctypes.c_int64),
                ("pad_slots", ctypes.c_int64), ("aux", ctypes.c_int64), ("params", Params)]


EXPORTED = [
    "spmv_status_str", "spmv_last_error", "spmv_mat_from_csr", "spmv_mat_from_coo", "spmv_convert", "spmv_to_csr",
    "spmv_array_bytes", "spmv_export", "spmv_mat_info", "spmv_mat_free", "spmv_run", "spmv_spmm",
    "spmv_batch_create", "spmv_batch_run", "spmv_batch_free", "spmv_time", "spmv_scrub", "spmv_copy_probe",
    "spmv_gather_probe",
    "spmv_autotune", "spmv_features", "spmv_model_create", "spmv_model_load", "spmv_model_save",
    "spmv_model_params", "spmv_model_free", "spmv_select", "spmv_mlp_forward", "spmv_mlp_backward", "spmv_mlp_adam",
    "spmv_scale_features", "spmv_feature_range", "spmv_mlp_train", "spmv_run_timed", "spmv_spmm_timed",
    "spmv_batch_run_timed", "spmv_autotune_cache_clear", "spmv_mem_in_use", "spmv_mem_release",
    "spmv_mlp_backward_noalloc",
]

_L = None


def lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: the HIP library must be built (__graft_entry__.build())")
        # torch first: it loads the HIP runtime it ships with, and the library
        # then binds to that one (same soname).  Loaded the other way round a
        # process would hold two HIP runtimes, and the second to initialise
        # finds no device.  (Importing torch does not touch the GPU.)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, vp, dp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_double
        st = ctypes.c_int
        sig = {
            "spmv_status_str": (ctypes.c_char_p, [st]),
            "spmv_last_error": (ctypes.c_char_p, []),
            "spmv_mat_from_csr": (st, [i64, i64, i64, vp, vp, vp, st, st, u32, vp, ctypes.POINTER(vp)]),
            "spmv_mat_from_coo": (st, [i64, i64, i64, vp, vp, vp, st, st, vp, ctypes.POINTER(vp)]),
            "spmv_convert": (st, [vp, st, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]),
            "spmv_to_csr": (st, [vp, vp, vp, vp, st, vp]),
            "spmv_array_bytes": (st, [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]),
            "spmv_export": (st, [vp, ctypes.c_char_p, vp, ctypes.c_size_t, vp]),
            "spmv_mat_info": (st, [vp, ctypes.POINTER(Info)]),
            "spmv_mat_free": (None, [vp]),
            "spmv_run": (st, [st, vp, vp, vp, vp]),
            "spmv_spmm": (st, [vp, vp, i64, vp, i64, i32, vp]),
            "spmv_batch_create": (st, [vp, i32, ctypes.POINTER(vp)]),
            "spmv_batch_run": (st, [vp, vp, vp, vp]),
            "spmv_batch_free": (None, [vp]),
            "spmv_time": (st, [st, vp, vp, vp, st, st, st, dp, i64, vp, vp]),
            "spmv_scrub": (st, [i64, vp]),
            "spmv_copy_probe": (st, [i64, st, vp, ctypes.POINTER(dp)]),
            "spmv_gather_probe": (st, [i64, i64, st, st, i64, vp, ctypes.POINTER(dp)]),
            "spmv_autotune": (st, [vp, st, vp, vp, i64, st, ctypes.POINTER(Params), ctypes.POINTER(dp), vp]),
            "spmv_features": (st, [vp, vp, vp]),
            "spmv_model_create": (st, [vp, vp, vp, ctypes.POINTER(vp)]),
            "spmv_model_load": (st, [ctypes.c_char_p, ctypes.POINTER(vp)]),
            "spmv_model_save": (st, [vp, ctypes.c_char_p]),
            "spmv_model_params": (st, [vp, vp, vp, vp]),
            "spmv_model_free": (None, [vp]),
            "spmv_select": (st, [vp, vp, ctypes.POINTER(st), vp]),
            "spmv_mlp_forward": (st, [vp, vp, i32, vp, vp, vp, vp]),
            "spmv_mlp_backward": (st, [vp, vp, vp, i32, vp, vp, vp]),
            "spmv_mlp_backward_noalloc": (st, [vp, vp, vp, i32, vp, vp, vp]),
            "spmv_mlp_adam": (st, [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, vp]),
            "spmv_scale_features": (st, [vp, i32, vp, vp, vp, vp]),
            "spmv_feature_range": (st, [vp, i32, vp, vp, vp]),
            "spmv_mlp_train": (st, [vp, vp, vp, i32, vp, i32, i32, ctypes.c_float, vp, vp]),
            "spmv_run_timed": (st, [st, vp, vp, vp, vp, vp, vp]),
            "spmv_spmm_timed": (st, [vp, vp, i64, vp, i64, i32, vp, vp, vp]),
            "spmv_batch_run_timed": (st, [vp, vp, vp, vp, vp, vp]),
            "spmv_autotune_cache_clear": (None, []),
            "spmv_mem_in_use": (i64, []),
            "spmv_mem_release": (i64, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _L = L
    return _L


def check(status: int):
    if status != 0:
        raise SpmvError(status, lib().spmv_last_error().decode(errors="replace"))


# ------------------------------------------------------------ plumbing

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the SpMV library runs on the device only")
    return torch


def stream():
    """The current torch (HIP) stream as a void*."""
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def timing_events():
    """A (start, stop) pair of timing-enabled torch events, created on the
    device (recorded once) so their handles can be passed to the timed runs."""
    torch = _torch()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    b.record()
    return a, b


def _ev(e):
    return ctypes.c_void_p(e.cuda_event)


def dptr(t):
    """Device pointer of a torch tensor (must be contiguous)."""
    assert t.is_cuda and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def hptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def np_dtype(dt: int):
    return np.float64 if dt == F64 else np.float32


def torch_dtype(dt: int):
    torch = _torch()
    return torch.float64 if dt == F64 else torch.float32


# ------------------------------------------------------------- matrices

class Matrix:
    """Owning wrapper of an spmv_mat_t handle."""

    def __init__(self, handle, keep=None):
        self.h = handle
        inf = Info()
        check(lib().spmv_mat_info(self.h, ctypes.byref(inf)))
        self.info = inf
        self.fmt = FMT_NAMES[inf.fmt]
        self.dtype = inf.dtype
        self.M, self.N, self.nnz = inf.M, inf.N, inf.nnz
        self._keep = keep

    def free(self):
        if getattr(self, "h", None):
            lib().spmv_mat_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # interpreter shutdown: module globals may already be gone
            pass

    @property
    def params(self) -> dict:
        return self.info.params.as_dict()

    # construction ------------------------------------------------------
    @staticmethod
    def from_csr(M, N, ptr, col, val, dtype=F64, check_cols=True) -> "Matrix":
        """From host numpy arrays (values cast to the dtype) or device tensors."""
        h = ctypes.c_void_p()
        flags = 0 if check_cols else 1
        if isinstance(ptr, np.ndarray):
            ptr = np.ascontiguousarray(ptr, np.int32)
            col = np.ascontiguousarray(col, np.int32)
            val = np.ascontiguousarray(val, np_dtype(dtype))
            check(lib().spmv_mat_from_csr(M, N, len(col), hptr(ptr), hptr(col), hptr(val), dtype, 0, flags,
                                          stream(), ctypes.byref(h)))
        else:
            check(lib().spmv_mat_from_csr(M, N, col.numel(), dptr(ptr), dptr(col), dptr(val), dtype, 1, flags,
                                          stream(), ctypes.byref(h)))
        return Matrix(h)

    @staticmethod
    def from_host(A, dtype=F64) -> "Matrix":
        return Matrix.from_csr(A.M, A.N, A.ptr, A.col, A.val, dtype)

    @staticmethod
    def from_coo(M, N, row, col, val, dtype=F64) -> "Matrix":
        h = ctypes.c_void_p()
        row = np.ascontiguousarray(row, np.int32)
        col = np.ascontiguousarray(col, np.int32)
        val = np.ascontiguousarray(val, np_dtype(dtype))
        check(lib().spmv_mat_from_coo(M, N, len(row), hptr(row), hptr(col), hptr(val), dtype, 0, stream(),
                                      ctypes.byref(h)))
        return Matrix(h)

    def convert(self, fmt: str, **kw) -> "Matrix":
        h = ctypes.c_void_p()
        p = params(**kw)
        check(lib().spmv_convert(self.h, FMT[fmt], ctypes.byref(p), stream(), ctypes.byref(h)))
        return Matrix(h)

    # inspection --------------------------------------------------------
    def to_csr(self):
        ptr = np.empty(self.M + 1, np.int32)
        col = np.empty(self.nnz, np.int32)
        val = np.empty(self.nnz, np_dtype(self.dtype))
        check(lib().spmv_to_csr(self.h, hptr(ptr), hptr(col), hptr(val), 0, stream()))
        return ptr, col, val

    def export(self, name: str, dtype) -> np.ndarray:
        n = ctypes.c_size_t()
        check(lib().spmv_array_bytes(self.h, name.encode(), ctypes.byref(n)))
        out = np.empty(n.value // np.dtype(dtype).itemsize, dtype)
        check(lib().spmv_export(self.h, name.encode(), hptr(out), n.value, stream()))
        return out

    # compute -----------------------------------------------------------
    def run(self, x, y=None):
        """y = A x on the current stream; x, y: device tensors of the dtype."""
        torch = _torch()
        if y is None:
            y = torch.empty(self.M, dtype=torch_dtype(self.dtype), device=x.device)
        check(lib().spmv_run(FMT[self.fmt], self.h, dptr(x), dptr(y), stream()))
        return y

    def run_timed(self, x, y, events):
        """As run; events = (start, stop) from timing_events() are recorded at
        the start of the run's first kernel and the end of its last."""
        check(lib().spmv_run_timed(FMT[self.fmt], self.h, dptr(x), dptr(y), stream(), _ev(events[0]),
                                   _ev(events[1])))
        return y

    def spmm_timed(self, X, Y, events):
        check(lib().spmv_spmm_timed(self.h, dptr(X), X.stride(0), dptr(Y), Y.stride(0), X.shape[1], stream(),
                                    _ev(events[0]), _ev(events[1])))
        return Y

    def spmm(self, X, Y=None):
        torch = _torch()
        k = X.shape[1]
        if Y is None:
            Y = torch.empty((self.M, k), dtype=torch_dtype(self.dtype), device=X.device)
        check(lib().spmv_spmm(self.h, dptr(X), X.stride(0), dptr(Y), Y.stride(0), k, stream()))
        return Y

    def time(self, x, y, warmup=5, min_reps=20, max_reps=1000, rel_ci=0.05, scrub_bytes=512 << 20) -> dict:
        out = (ctypes.c_double * 5)()
        check(lib().spmv_time(FMT[self.fmt], self.h, dptr(x), dptr(y), warmup, min_reps, max_reps, rel_ci,
                              scrub_bytes, stream(), out))
        return dict(median_ms=out[0], mean_ms=out[1], ci_ms=out[2], reps=int(out[3]), min_ms=out[4])

    def features(self) -> np.ndarray:
        f = np.empty(12, np.float64)
        check(lib().spmv_features(self.h, hptr(f), stream()))
        return f

    def autotune(self, fmt: str, x, y, scrub_bytes=512 << 20, reps=10, **kw):
        p = params(**kw)
        ms = ctypes.c_double()
        check(lib().spmv_autotune(self.h, FMT[fmt], dptr(x), dptr(y), scrub_bytes, reps, ctypes.byref(p),
                                  ctypes.byref(ms), stream()))
        return p.as_dict(), ms.value


def scrub(nbytes=512 << 20):
    check(lib().spmv_scrub(nbytes, stream()))


def copy_probe(nbytes=1 << 30, reps=20) -> float:
    g = ctypes.c_double()
    check(lib().spmv_copy_probe(nbytes, reps, stream(), ctypes.byref(g)))
    return g.value


def gather_probe(nx: int, rows: int, dtype: int = F64, reps: int = 10, scrub_bytes: int = 512 << 20) -> float:
    """Median ms of a balanced 16-per-row SpMV with uniformly random columns
    over an x of nx values: the floor for 16 * rows scattered gathers."""
    ms = ctypes.c_double()
    check(lib().spmv_gather_probe(int(nx), int(rows), int(dtype), int(reps), int(scrub_bytes), stream(),
                                  ctypes.byref(ms)))
    return ms.value


# -------------------------------------------------------------- batches

class Batch:
    def __init__(self, mats):
        self.mats = list(mats)
        arr = (ctypes.c_void_p * len(self.mats))(*[m.h for m in self.mats])
        self.h = ctypes.c_void_p()
        check(lib().spmv_batch_create(arr, len(self.mats), ctypes.byref(self.h)))

    def run(self, xs, ys, events=None):
        xa = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * len(ys))(*[y.data_ptr() for y in ys])
        if events is None:
            check(lib().spmv_batch_run(self.h, xa, ya, stream()))
        else:
            check(lib().spmv_batch_run_timed(self.h, xa, ya, stream(), _ev(events[0]), _ev(events[1])))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().spmv_batch_free(self.h)
                self.h = None
        except Exception:
            pass


# ---------------------------------------------------------------- model

class Model:
    def __init__(self, handle):
        self.h = handle

    @staticmethod
    def create(params: np.ndarray, fmin, fmax) -> "Model":
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == NPARAM
        lo = np.ascontiguousarray(fmin, np.float64)
        hi = np.ascontiguousarray(fmax, np.float64)
        h = ctypes.c_void_p()
        check(lib().spmv_model_create(hptr(p), hptr(lo), hptr(hi), ctypes.byref(h)))
        return Model(h)

    @staticmethod
    def load(path: str) -> "Model":
        h = ctypes.c_void_p()
        check(lib().spmv_model_load(path.encode(), ctypes.byref(h)))
        return Model(h)

    def save(self, path: str):
        check(lib().spmv_model_save(self.h, path.encode()))

    def params(self):
        p = np.empty(NPARAM, np.float32)
        lo = np.empty(12)
        hi = np.empty(12)
        check(lib().spmv_model_params(self.h, hptr(p), hptr(lo), hptr(hi)))
        return p, lo, hi

    def select(self, features) -> tuple[str, np.ndarray]:
        f = np.ascontiguousarray(features, np.float64)
        best = ctypes.c_int()
        sc = np.empty(5, np.float32)
        check(lib().spmv_select(self.h, hptr(f), ctypes.byref(best), hptr(sc)))
        return FMT_NAMES[best.value], sc

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().spmv_model_free(self.h)
                self.h = None
        except Exception:
            pass

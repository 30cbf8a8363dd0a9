"""ctypes binding of libapo.so (the C ABI declared in include/apo.h).

Argument marshalling only: every step of the optimiser runs in the HIP
kernels behind the ABI.  PyTorch supplies the device workspace and the
stream the library launches on.  There is no fallback: if the library is
missing or cannot be loaded, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapo.so")

APO_OK, APO_E_INVAL, APO_E_NOMEM, APO_E_DEVICE, APO_E_DONE, APO_E_STATE, APO_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
APO_FP64, APO_FP32, APO_BF16 = 0, 1, 2
KINDS = {"sphere": 0, "rastrigin": 1, "rosenbrock": 2, "ackley": 3, "kapur": 4, "otsu": 5}
APO_FLAG_TRACE = 1
APO_FLAG_PDR_PLUS = 2
OPS = {0: "dormancy", 1: "reproduction", 2: "autotroph", 3: "heterotroph"}


class Objective(C.Structure):
    _fields_ = [("kind", C.c_int32), ("shift", C.POINTER(C.c_double)),
                ("rot", C.POINTER(C.c_double)), ("hist", C.POINTER(C.c_uint64))]


class Options(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("precision", C.c_int32), ("objective", Objective),
                ("run_id", C.c_uint32), ("flags", C.c_uint32), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class RunDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lb", C.POINTER(C.c_double)), ("ub", C.POINTER(C.c_double)),
                ("pop", C.c_int32), ("np", C.c_int32), ("pf_max", C.c_double),
                ("seed", C.c_uint64), ("opt", Options)]


class BatchOptions(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class APOError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def lib():
    """The loaded libapo.so (loaded once, after torch so both share one HIP
    runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no non-HIP fallback)")
    try:
        import torch  # noqa: F401  (load torch's HIP runtime first)
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, d, i32, u64, vp = C.POINTER, C.c_double, C.c_int32, C.c_uint64, C.c_void_p
    L.apo_workspace_bytes.restype = C.c_size_t
    L.apo_workspace_bytes.argtypes = [i32, i32, P(Options)]
    L.apo_create.restype = C.c_int
    L.apo_create.argtypes = [i32, P(d), P(d), i32, i32, d, u64, P(Options), P(vp)]
    for name in ("apo_step", "apo_destroy"):
        getattr(L, name).restype = C.c_int
        getattr(L, name).argtypes = [vp]
    L.apo_run.restype = C.c_int
    L.apo_run.argtypes = [vp, i32]
    L.apo_best.restype = C.c_int
    L.apo_best.argtypes = [vp, P(d), P(d), P(C.c_int64)]
    L.apo_info.restype = C.c_int
    L.apo_info.argtypes = [vp, P(i32), P(C.c_int64)]
    L.apo_get_state.restype = C.c_int
    L.apo_get_state.argtypes = [vp, P(d), P(d), P(i32)]
    L.apo_set_state.restype = C.c_int
    L.apo_set_state.argtypes = [vp, P(d), P(d), i32]
    L.apo_get_trace.restype = C.c_int
    L.apo_get_trace.argtypes = [vp, P(d), P(d), P(i32), P(i32)]
    L.apo_time_kernels.restype = C.c_int
    L.apo_time_kernels.argtypes = [vp, i32, P(d)]
    L.apo_histogram_u8.restype = C.c_int
    L.apo_histogram_u8.argtypes = [vp, u64, vp, vp]
    L.apo_histogram_u8_noalloc.restype = C.c_int
    L.apo_histogram_u8_noalloc.argtypes = [vp, u64, vp, vp]
    L.apo_batch_workspace_bytes.restype = C.c_size_t
    L.apo_batch_workspace_bytes.argtypes = [i32, P(RunDesc)]
    L.apo_batch_create.restype = C.c_int
    L.apo_batch_create.argtypes = [i32, P(RunDesc), P(BatchOptions), P(vp)]
    L.apo_batch_run.restype = C.c_int
    L.apo_batch_run.argtypes = [vp, i32]
    L.apo_batch_member.restype = C.c_int
    L.apo_batch_member.argtypes = [vp, i32, P(vp)]
    L.apo_batch_tune.restype = C.c_int
    L.apo_batch_tune.argtypes = [vp, i32, P(i32), P(d)]
    L.apo_batch_destroy.restype = C.c_int
    L.apo_batch_destroy.argtypes = [vp]
    L.apo_time_gemm_stages.restype = C.c_int
    L.apo_time_gemm_stages.argtypes = [vp, i32, P(d)]
    L.apo_precision_stats.restype = C.c_int
    L.apo_precision_stats.argtypes = [vp, P(C.c_int64), P(C.c_int64)]
    L.apo_strerror.restype = C.c_char_p
    L.apo_strerror.argtypes = [C.c_int]
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().apo_strerror(int(status)).decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise APOError(rc, what)
    return rc


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))

"""MI355X (gfx950) Artificial Protozoa Optimizer population step.

``APO`` wraps one handle of libapo.so: creation (Algorithm 1's input and
initial population), ``step`` / ``run`` (the per-iteration population step:
sort, Dr, Eqs. (1)-(13), clamp, evaluation, greedy selection), ``best``
(Algorithm 1's output), checkpoint/trace hooks and per-kernel timing.
``histogram_u8`` reduces an 8-bit image on the GPU for the thresholding
objectives.  PyTorch provides the device workspace and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from ._lib import (APO_E_DONE, APO_FLAG_TRACE, APO_FP32, APO_FP64, KINDS, OPS, APOError,
                   Objective, Options, _check, _dptr, lib, strerror)

__all__ = ["APO", "APOError", "histogram_u8", "workspace_bytes", "lib", "strerror", "OPS"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libapo needs a HIP device; none is visible")
    return torch


def _options(max_iter, precision, kind, shift, rot, hist, run_id, flags, stream=None,
             workspace=None, workspace_bytes=0):
    o = Options()
    o.max_iter = int(max_iter)
    o.precision = APO_FP32 if precision in ("fp32", APO_FP32) else APO_FP64
    o.objective.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
    o.objective.shift = _dptr(shift)
    o.objective.rot = _dptr(rot)
    o.objective.hist = None if hist is None else hist.ctypes.data_as(C.POINTER(C.c_uint64))
    o.run_id = int(run_id)
    o.flags = int(flags)
    o.stream = stream
    o.workspace = workspace
    o.workspace_bytes = int(workspace_bytes)
    return o


def workspace_bytes(dim, pop, np_pairs=1, max_iter=1, precision="fp64", kind="sphere",
                    rotated=False, trace=False) -> int:
    rot = np.eye(dim) if rotated else None
    hist = np.ones(256, np.uint64) if kind in ("kapur", "otsu") else None
    o = _options(max_iter, precision, kind, None, rot, hist, 0, APO_FLAG_TRACE if trace else 0)
    return int(lib().apo_workspace_bytes(int(dim), int(pop), int(np_pairs), C.byref(o)))


class APO:
    """One optimiser handle.

    Parameters follow ``apo_create``: dim, lb, ub (scalars or [dim]), pop,
    np_pairs, pf_max, seed, max_iter, precision ("fp64" | "fp32"), objective
    kind and its inputs (shift [dim], rot [dim, dim] row-major, hist [256]).
    ``trace=True`` keeps every candidate of the last step for
    ``get_trace``.  The workspace is a torch uint8 tensor on the current
    device and launches go to ``stream`` (default: torch's current stream).
    """

    def __init__(self, dim, lb, ub, pop, np_pairs=1, pf_max=0.1, seed=1, max_iter=100,
                 precision="fp64", kind="sphere", shift=None, rot=None, hist=None, run_id=0,
                 trace=False, stream=None):
        torch = _torch()
        self.dim, self.pop, self.max_iter = int(dim), int(pop), int(max_iter)
        self.precision = precision
        lb = np.ascontiguousarray(np.broadcast_to(np.asarray(lb, np.float64), (self.dim,)))
        ub = np.ascontiguousarray(np.broadcast_to(np.asarray(ub, np.float64), (self.dim,)))
        shift = None if shift is None else np.ascontiguousarray(shift, np.float64).reshape(self.dim)
        rot = None if rot is None else np.ascontiguousarray(rot, np.float64).reshape(self.dim, self.dim)
        hist = None if hist is None else np.ascontiguousarray(hist, np.uint64).reshape(256)
        flags = APO_FLAG_TRACE if trace else 0
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        o = _options(max_iter, precision, kind, shift, rot, hist, run_id, flags)
        nbytes = int(lib().apo_workspace_bytes(self.dim, self.pop, int(np_pairs), C.byref(o)))
        if nbytes == 0:
            raise APOError(-1, "apo_workspace_bytes")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=torch.cuda.current_device())
        o = _options(max_iter, precision, kind, shift, rot, hist, run_id, flags,
                     stream=C.c_void_p(self._stream.cuda_stream),
                     workspace=C.c_void_p(self._ws.data_ptr()), workspace_bytes=nbytes)
        h = C.c_void_p()
        _check(lib().apo_create(self.dim, _dptr(lb), _dptr(ub), self.pop, int(np_pairs),
                                float(pf_max), int(seed) & (2**64 - 1), C.byref(o), C.byref(h)),
               "apo_create")
        self._h = h

    # -- life cycle -----------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().apo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the step -------------------------------------------------------
    def step(self) -> bool:
        """One iteration; False once the budget is spent."""
        rc = lib().apo_step(self._h)
        if rc == APO_E_DONE:
            return False
        _check(rc, "apo_step")
        return True

    def run(self, iters: Optional[int] = None) -> int:
        n = self.max_iter if iters is None else int(iters)
        return _check(lib().apo_run(self._h, n), "apo_run")

    def time_kernels(self, iters: int):
        out = np.zeros(2)
        n = _check(lib().apo_time_kernels(self._h, int(iters), _dptr(out)), "apo_time_kernels")
        return n, {"rank_us": float(out[0]), "step_us": float(out[1])}

    # -- results --------------------------------------------------------
    def best(self):
        x = np.zeros(self.dim)
        f = C.c_double()
        fes = C.c_int64()
        _check(lib().apo_best(self._h, _dptr(x), C.byref(f), C.byref(fes)), "apo_best")
        return x, f.value, fes.value

    def info(self):
        it = C.c_int32()
        fes = C.c_int64()
        _check(lib().apo_info(self._h, C.byref(it), C.byref(fes)), "apo_info")
        return it.value, fes.value

    def get_state(self):
        X = np.zeros((self.pop, self.dim))
        F = np.zeros(self.pop)
        it = C.c_int32()
        _check(lib().apo_get_state(self._h, _dptr(X), _dptr(F), C.byref(it)), "apo_get_state")
        return X, F, it.value

    def set_state(self, X, F, iteration: int):
        X = np.ascontiguousarray(X, np.float64).reshape(self.pop, self.dim)
        F = np.ascontiguousarray(F, np.float64).reshape(self.pop)
        _check(lib().apo_set_state(self._h, _dptr(X), _dptr(F), int(iteration)), "apo_set_state")

    def get_trace(self):
        Y = np.zeros((self.pop, self.dim))
        Fy = np.zeros(self.pop)
        op = np.zeros(self.pop, np.int32)
        perm = np.zeros(self.pop, np.int32)
        _check(lib().apo_get_trace(self._h, _dptr(Y), _dptr(Fy),
                                   op.ctypes.data_as(C.POINTER(C.c_int32)),
                                   perm.ctypes.data_as(C.POINTER(C.c_int32))), "apo_get_trace")
        return Y, Fy, op, perm


def histogram_u8(img, stream=None):
    """256-bin histogram (uint32 counts, device tensor) of a uint8 device
    tensor, computed by the library's histogram kernel."""
    torch = _torch()
    if img.dtype != torch.uint8 or not img.is_cuda:
        raise ValueError("histogram_u8 needs a uint8 device tensor")
    img = img.contiguous()
    out = torch.empty(256, dtype=torch.int32, device=img.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().apo_histogram_u8(C.c_void_p(img.data_ptr()), img.numel(),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)),
           "apo_histogram_u8")
    return out

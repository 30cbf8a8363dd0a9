"""MI355X (gfx950) Artificial Protozoa Optimizer population step.

``APO`` wraps one handle of libapo.so: creation (Algorithm 1's input and
initial population), ``step`` / ``run`` (the per-iteration population step:
sort, Dr, Eqs. (1)-(13), clamp, evaluation, greedy selection), ``best``
(Algorithm 1's output), checkpoint/trace hooks and per-kernel timing.
``histogram_u8`` reduces an 8-bit image on the GPU for the thresholding
objectives.  ``Batch`` advances many independent runs together (one launch
per kernel shape per iteration) and hands out each run as a non-owning
``APO`` view.  PyTorch provides the device workspace and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from ._lib import (APO_BF16, APO_E_DONE, APO_FLAG_PDR_PLUS, APO_FLAG_TRACE,
                   APO_FP32, APO_FP64,
                   KINDS,
                   OPS, APOError,
                   BatchOptions, Objective, Options, RunDesc, _check, _dptr, lib, strerror)

__all__ = ["APO", "APOError", "Batch", "histogram_u8", "histogram_u8_noalloc", "workspace_bytes", "lib", "strerror",
           "OPS"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libapo needs a HIP device; none is visible")
    return torch


def _options(max_iter, precision, kind, shift, rot, hist, run_id, flags, stream=None,
             workspace=None, workspace_bytes=0):
    o = Options()
    o.max_iter = int(max_iter)
    o.precision = {"fp64": APO_FP64, "fp32": APO_FP32, "bf16": APO_BF16}.get(precision, precision)
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
    return int(lib().apo_workspace_bytes(int(dim), int(pop), C.byref(o)))


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
                 trace=False, stream=None, pdr_plus=False):
        torch = _torch()
        self.dim, self.pop, self.max_iter = int(dim), int(pop), int(max_iter)
        self.precision = precision
        lb = np.ascontiguousarray(np.broadcast_to(np.asarray(lb, np.float64), (self.dim,)))
        ub = np.ascontiguousarray(np.broadcast_to(np.asarray(ub, np.float64), (self.dim,)))
        shift = None if shift is None else np.ascontiguousarray(shift, np.float64).reshape(self.dim)
        rot = None if rot is None else np.ascontiguousarray(rot, np.float64).reshape(self.dim, self.dim)
        hist = None if hist is None else np.ascontiguousarray(hist, np.uint64).reshape(256)
        flags = (APO_FLAG_TRACE if trace else 0) | (APO_FLAG_PDR_PLUS if pdr_plus else 0)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        o = _options(max_iter, precision, kind, shift, rot, hist, run_id, flags)
        nbytes = int(lib().apo_workspace_bytes(self.dim, self.pop, C.byref(o)))
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

    @classmethod
    def _view(cls, handle, dim, pop, max_iter, precision, owner):
        """A batch member: same calls, no ownership (the batch frees it)."""
        v = cls.__new__(cls)
        v.dim, v.pop, v.max_iter, v.precision = int(dim), int(pop), int(max_iter), precision
        v._h = handle
        v._owner = owner
        return v

    # -- life cycle -----------------------------------------------------
    def close(self):
        if getattr(self, "_owner", None) is not None:   # a batch member
            self._h = None
            return
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
        """Up to ``iters`` iterations (default: the rest of the budget) as
        replayed graphs; ``run(0)`` only captures the graphs."""
        n = self.max_iter if iters is None else int(iters)
        return _check(lib().apo_run(self._h, n), "apo_run")

    def time_kernels(self, iters: int):
        out = np.zeros(2)
        n = _check(lib().apo_time_kernels(self._h, int(iters), _dptr(out)), "apo_time_kernels")
        return n, {"rank_us": float(out[0]), "step_us": float(out[1])}

    def time_gemm_stages(self, iters: int):
        """Per-stage microseconds per iteration of the GEMM form."""
        out = np.zeros(6)
        n = _check(lib().apo_time_gemm_stages(self._h, int(iters), _dptr(out)),
                   "apo_time_gemm_stages")
        names = ("candidates", "product", "classify", "rescore_product", "select", "sort")
        return n, dict(zip(names, map(float, out)))

    def precision_stats(self):
        """(candidates re-scored in binary32, candidates estimated) of the
        BF16 form."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().apo_precision_stats(self._h, C.byref(a), C.byref(b)), "apo_precision_stats")
        return a.value, b.value

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


class Batch:
    """Independent runs advanced together (``apo_batch_*``).

    ``runs`` is a list of dicts with the keyword arguments of ``APO``
    (dim, lb, ub, pop, np_pairs, pf_max, seed, max_iter, precision, kind,
    shift, rot, hist, run_id, trace).  ``batch[i]`` is run i as an ``APO``
    view (best, info, get_state, set_state, get_trace); ``run(n)`` steps
    every run; ``tune(n)`` picks the launch schedule.
    """

    def __init__(self, runs, stream=None):
        torch = _torch()
        self._keep = []
        self._specs = []
        n = len(runs)
        descs = (RunDesc * n)()
        for i, r in enumerate(runs):
            dim = int(r["dim"])
            lb = np.ascontiguousarray(np.broadcast_to(np.asarray(r["lb"], np.float64), (dim,)))
            ub = np.ascontiguousarray(np.broadcast_to(np.asarray(r["ub"], np.float64), (dim,)))
            shift = r.get("shift")
            shift = None if shift is None else np.ascontiguousarray(shift, np.float64).reshape(dim)
            rot = r.get("rot")
            rot = None if rot is None else np.ascontiguousarray(rot, np.float64).reshape(dim, dim)
            hist = r.get("hist")
            hist = None if hist is None else np.ascontiguousarray(hist, np.uint64).reshape(256)
            self._keep += [lb, ub, shift, rot, hist]
            prec = r.get("precision", "fp64")
            d = descs[i]
            d.dim = dim
            d.lb, d.ub = _dptr(lb), _dptr(ub)
            d.pop = int(r["pop"])
            d.np = int(r.get("np_pairs", 1))
            d.pf_max = float(r.get("pf_max", 0.1))
            d.seed = int(r.get("seed", 1)) & (2**64 - 1)
            d.opt = _options(r.get("max_iter", 100), prec, r.get("kind", "sphere"), shift, rot,
                             hist, r.get("run_id", 0), APO_FLAG_TRACE if r.get("trace") else 0)
            self._specs.append((dim, d.pop, int(r.get("max_iter", 100)), prec))
        nbytes = int(lib().apo_batch_workspace_bytes(n, descs))
        if nbytes == 0:
            raise APOError(-1, "apo_batch_workspace_bytes")
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=torch.cuda.current_device())
        o = BatchOptions()
        o.stream = C.c_void_p(self._stream.cuda_stream)
        o.workspace = C.c_void_p(self._ws.data_ptr())
        o.workspace_bytes = nbytes
        b = C.c_void_p()
        _check(lib().apo_batch_create(n, descs, C.byref(o), C.byref(b)), "apo_batch_create")
        self._b = b
        self._members = []
        for i in range(n):
            h = C.c_void_p()
            _check(lib().apo_batch_member(b, i, C.byref(h)), "apo_batch_member")
            self._members.append(APO._view(h, *self._specs[i], owner=self))

    def __len__(self):
        return len(self._members)

    def __getitem__(self, i):
        return self._members[i]

    def run(self, iters: int) -> int:
        return _check(lib().apo_batch_run(self._b, int(iters)), "apo_batch_run")

    def tune(self, iters: int = 16):
        sched = C.c_int32()
        us = np.zeros(4)
        _check(lib().apo_batch_tune(self._b, int(iters), C.byref(sched), _dptr(us)),
               "apo_batch_tune")
        return sched.value, us

    def close(self):
        if getattr(self, "_b", None):
            for m in self._members:
                m._h = None
            lib().apo_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def histogram_u8(img, stream=None) -> np.ndarray:
    """256-bin histogram (numpy uint64 counts) of a uint8 device tensor,
    computed by the library's histogram kernel (``apo_histogram_u8``)."""
    torch = _torch()
    if img.dtype != torch.uint8 or not img.is_cuda:
        raise ValueError("histogram_u8 needs a uint8 device tensor")
    img = img.contiguous()
    out = np.zeros(256, dtype=np.uint64)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().apo_histogram_u8(C.c_void_p(img.data_ptr()), img.numel(),
                                  out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                  C.c_void_p(s.cuda_stream)), "apo_histogram_u8")
    return out


def histogram_u8_noalloc(img, out, stream=None):
    """The allocation-free histogram (``apo_histogram_u8_noalloc``): counts
    of a uint8 device tensor into ``out``, a device int64/uint64 tensor of
    256 elements; asynchronous on ``stream`` (default: the current stream)."""
    torch = _torch()
    if img.dtype != torch.uint8 or not img.is_cuda or not img.is_contiguous():
        raise ValueError("histogram_u8_noalloc needs a contiguous uint8 device tensor")
    if (not out.is_cuda or out.numel() != 256 or not out.is_contiguous()
            or out.dtype not in (torch.int64, torch.uint64)):
        raise ValueError("histogram_u8_noalloc needs a contiguous 256-element 64-bit device output")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().apo_histogram_u8_noalloc(C.c_void_p(img.data_ptr()), img.numel(),
                                          C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)),
           "apo_histogram_u8_noalloc")
    return out

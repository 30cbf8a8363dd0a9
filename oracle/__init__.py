"""ctypes wrapper around the plain FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
code with the HIP path.  See ``apo_oracle.c`` for what each entry point
follows in the paper (Section 3, Eqs. (1)-(13); Algorithm 1; the worked
example of Section 4.1).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import build as _build

KIND = {"sphere": 0, "rastrigin": 1, "rosenbrock": 2, "ackley": 3, "kapur": 4, "otsu": 5}
OPS = {0: "dormancy", 1: "reproduction", 2: "autotroph", 3: "heterotroph"}


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("pop", C.c_int32), ("np", C.c_int32), ("max_iter", C.c_int32),
        ("pf_max", C.c_double), ("seed", C.c_uint64), ("run", C.c_uint32), ("kind", C.c_int32),
        ("lb", C.POINTER(C.c_double)), ("ub", C.POINTER(C.c_double)),
        ("shift", C.POINTER(C.c_double)), ("rot", C.POINTER(C.c_double)),
        ("hist", C.POINTER(C.c_uint64)), ("pdr_plus", C.c_int32),
    ]


class _Trace(C.Structure):
    _fields_ = [
        ("Y", C.POINTER(C.c_double)), ("Fy", C.POINTER(C.c_double)),
        ("op", C.POINTER(C.c_int32)), ("perm", C.POINTER(C.c_int32)),
        ("mcount", C.POINTER(C.c_int32)), ("nb", C.POINTER(C.c_int32)),
        ("accepted", C.POINTER(C.c_uint8)), ("dr_count", C.POINTER(C.c_int32)),
    ]


_lib = None


class _Draws(C.Structure):
    """One rank's draws for ``oracle_step_scripted`` (``oracle_draws``)."""
    _fields_ = [
        ("in_dr", C.c_int32), ("u_op", C.c_double), ("u_f", C.c_double), ("u_rep", C.c_double),
        ("sgn", C.c_double), ("j", C.c_int32), ("km", C.c_int32 * 8), ("kp", C.c_int32 * 8),
        ("mask", C.POINTER(C.c_uint8)), ("U", C.POINTER(C.c_double)),
    ]


def _configure(L):
    P = C.POINTER
    L.oracle_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.oracle_uniform.restype = C.c_double
    L.oracle_uniform.argtypes = [C.c_uint32]
    L.oracle_bounded.restype = C.c_uint32
    L.oracle_bounded.argtypes = [C.c_uint32, C.c_uint32]
    L.oracle_subset_pi.restype = C.c_uint32
    L.oracle_subset_pi.argtypes = [C.c_uint32, C.c_uint32, P(C.c_uint32)]
    L.oracle_subset_mask.argtypes = [C.c_uint32, C.c_uint32, P(C.c_uint32), P(C.c_uint8)]
    L.oracle_objective.restype = C.c_double
    L.oracle_objective.argtypes = [P(_Problem), P(C.c_double)]
    L.oracle_rank_order.argtypes = [C.c_int32, P(C.c_double), P(C.c_int32)]
    L.oracle_init.argtypes = [P(_Problem), P(C.c_double), P(C.c_double)]
    L.oracle_finish.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(C.c_double),
                                P(C.c_double), P(C.c_uint8)]
    L.oracle_step.restype = C.c_int
    L.oracle_step.argtypes = [P(_Problem), C.c_int32, P(C.c_double), P(C.c_double), P(_Trace)]
    L.oracle_step_scripted.restype = C.c_int
    L.oracle_step_scripted.argtypes = [P(_Problem), C.c_int32, P(C.c_double), P(C.c_double),
                                       P(_Draws), P(_Trace)]
    L.oracle_best.restype = C.c_int32
    L.oracle_best.argtypes = [C.c_int32, P(C.c_double)]
    L.oracle_run.restype = C.c_int32
    L.oracle_run.argtypes = [P(_Problem), C.c_int32, C.c_int32, P(C.c_double), P(C.c_double)]
    L.oracle_histogram_u8.argtypes = [P(C.c_uint8), C.c_uint64, P(C.c_uint64)]
    if hasattr(L, "oracle_set_threads"):
        L.oracle_set_threads.restype = C.c_int32
        L.oracle_set_threads.argtypes = [C.c_int32]
        L.oracle_set_threads(1)
    return L


def load(path: str):
    """A separately built copy of the oracle (used by the tests that check
    the pins reject deliberately altered copies of the oracle source)."""
    return _configure(C.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = _configure(C.CDLL(_build.LIB))
    return _lib


def set_threads(n: int) -> int:
    """Spread the oracle's loops over protozoa across n threads (results are
    bit-identical for every n); returns the count in effect."""
    return int(lib().oracle_set_threads(int(n)))


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return C.POINTER(ctype)()
    return a.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def uniform(w: int) -> float:
    return lib().oracle_uniform(int(w))


def bounded(w: int, n: int) -> int:
    return lib().oracle_bounded(int(w), int(n))


def subset_pi(x: int, n: int, keys) -> int:
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    assert k.shape == (8,)
    return lib().oracle_subset_pi(int(x), int(n), _ptr(k, C.c_uint32))


def subset_mask(n: int, m: int, keys) -> list:
    """Members (ascending) of the coordinate-mask m-subset of [0, n)."""
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    assert k.shape == (8,) and n >= 1
    out = np.zeros(n, dtype=np.uint8)
    lib().oracle_subset_mask(int(n), int(m), _ptr(k, C.c_uint32), _ptr(out, C.c_uint8))
    return [int(x) for x in np.flatnonzero(out)]


def rank_order(F) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.float64)
    perm = np.zeros(F.shape[0], dtype=np.int32)
    lib().oracle_rank_order(F.shape[0], _ptr(F, C.c_double), _ptr(perm, C.c_int32))
    return perm


def best(F) -> int:
    F = np.ascontiguousarray(F, dtype=np.float64)
    return int(lib().oracle_best(F.shape[0], _ptr(F, C.c_double)))


def histogram_u8(img) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8).reshape(-1)
    h = np.zeros(256, dtype=np.uint64)
    lib().oracle_histogram_u8(_ptr(img, C.c_uint8), img.size, _ptr(h, C.c_uint64))
    return h


@dataclass
class StepTrace:
    Y: np.ndarray
    Fy: np.ndarray
    op: np.ndarray
    perm: np.ndarray
    mcount: np.ndarray
    nb: np.ndarray
    accepted: np.ndarray
    dr_count: int


@dataclass
class Problem:
    """An APO problem as the oracle sees it (all arrays FP64, copied)."""
    dim: int
    pop: int
    lb: np.ndarray
    ub: np.ndarray
    np_pairs: int = 1
    max_iter: int = 100
    pf_max: float = 0.1
    seed: int = 1
    run_id: int = 0
    kind: str = "sphere"
    shift: Optional[np.ndarray] = None
    rot: Optional[np.ndarray] = None
    hist: Optional[np.ndarray] = None
    pdr_plus: bool = False          # Eq. (13) with the opposite sign (a variant)
    lib: object = field(default=None, repr=False)   # None: the built oracle
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        self.lb = np.ascontiguousarray(np.broadcast_to(self.lb, (self.dim,)), dtype=np.float64)
        self.ub = np.ascontiguousarray(np.broadcast_to(self.ub, (self.dim,)), dtype=np.float64)
        if self.shift is not None:
            self.shift = np.ascontiguousarray(self.shift, dtype=np.float64).reshape(self.dim)
        if self.rot is not None:
            self.rot = np.ascontiguousarray(self.rot, dtype=np.float64).reshape(self.dim, self.dim)
        if self.hist is not None:
            self.hist = np.ascontiguousarray(self.hist, dtype=np.uint64).reshape(256)
        if self.kind in ("kapur", "otsu"):
            if self.hist is None:
                raise ValueError("histogram objectives need a histogram")
            if self.lb.min() < 0 or self.ub.max() > 255:
                raise ValueError("threshold bounds must lie in [0, 255]")

    def _lib(self):
        return self.lib if self.lib is not None else lib()

    def _c(self) -> _Problem:
        s = _Problem()
        s.dim, s.pop, s.np, s.max_iter = self.dim, self.pop, self.np_pairs, self.max_iter
        s.pf_max, s.seed, s.run, s.kind = self.pf_max, self.seed, self.run_id, KIND[self.kind]
        s.lb, s.ub = _ptr(self.lb, C.c_double), _ptr(self.ub, C.c_double)
        s.shift = _ptr(self.shift, C.c_double)
        s.rot = _ptr(self.rot, C.c_double)
        s.hist = _ptr(self.hist, C.c_uint64)
        s.pdr_plus = 1 if self.pdr_plus else 0
        return s

    # -- method ---------------------------------------------------------
    def objective(self, x) -> float:
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.dim)
        s = self._c()
        return self._lib().oracle_objective(C.byref(s), _ptr(x, C.c_double))

    def init(self):
        X = np.zeros((self.pop, self.dim))
        F = np.zeros(self.pop)
        s = self._c()
        self._lib().oracle_init(C.byref(s), _ptr(X, C.c_double), _ptr(F, C.c_double))
        return X, F

    def finish(self, X, F, Y):
        """Clamp, evaluate and greedily select (worked example, Step 6)."""
        X = np.array(X, dtype=np.float64, order="C")
        F = np.array(F, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64, order="C")
        Fy = np.zeros(self.pop)
        acc = np.zeros(self.pop, dtype=np.uint8)
        s = self._c()
        self._lib().oracle_finish(C.byref(s), _ptr(X, C.c_double), _ptr(F, C.c_double),
                            _ptr(Y, C.c_double), _ptr(Fy, C.c_double), _ptr(acc, C.c_uint8))
        return X, F, Y, Fy, acc.astype(bool)

    def _trace(self):
        nbw = 1 + 2 * self.np_pairs
        tr = StepTrace(Y=np.zeros((self.pop, self.dim)), Fy=np.zeros(self.pop),
                       op=np.zeros(self.pop, np.int32), perm=np.zeros(self.pop, np.int32),
                       mcount=np.zeros(self.pop, np.int32),
                       nb=np.zeros((self.pop, nbw), np.int32),
                       accepted=np.zeros(self.pop, np.uint8), dr_count=0)
        drc = np.zeros(1, np.int32)
        c_tr = _Trace(_ptr(tr.Y, C.c_double), _ptr(tr.Fy, C.c_double),
                      _ptr(tr.op, C.c_int32), _ptr(tr.perm, C.c_int32),
                      _ptr(tr.mcount, C.c_int32), _ptr(tr.nb, C.c_int32),
                      _ptr(tr.accepted, C.c_uint8), _ptr(drc, C.c_int32))
        return tr, c_tr, drc

    def step(self, t, X, F, trace: bool = True):
        """Iteration t (1-based) from state (X, F); returns (X', F', trace)."""
        X = np.array(X, dtype=np.float64, order="C")
        F = np.array(F, dtype=np.float64)
        tr = c_tr = drc = None
        if trace:
            tr, c_tr, drc = self._trace()
        s = self._c()
        rc = self._lib().oracle_step(C.byref(s), int(t), _ptr(X, C.c_double),
                                     _ptr(F, C.c_double),
                                     C.byref(c_tr) if c_tr is not None else None)
        if rc != 0:
            raise ValueError(f"oracle_step rejected t={t}")
        if tr is not None:
            tr.dr_count = int(drc[0])
            tr.accepted = tr.accepted.astype(bool)
        return X, F, tr

    def step_scripted(self, t, X, F, draws):
        """Iteration t with every random value supplied instead of drawn.

        ``draws[r]`` (r = 0-based rank after the sort) is a dict with keys
        in_dr (bool), u_op, u_f, u_rep, sgn (+1 / -1), j, km, kp (lists of
        np ranks), mask (D zeros / ones) and U (D values in (0, 1)); missing
        keys default to 0 (empty mask).  Returns (X', F', trace)."""
        if len(draws) != self.pop:
            raise ValueError("one draw record per rank")
        X = np.array(X, dtype=np.float64, order="C")
        F = np.array(F, dtype=np.float64)
        recs = (_Draws * self.pop)()
        keep = []
        for r, d in enumerate(draws):
            c = recs[r]
            c.in_dr = 1 if d.get("in_dr", False) else 0
            c.u_op, c.u_f = float(d.get("u_op", 0.0)), float(d.get("u_f", 0.0))
            c.u_rep, c.sgn = float(d.get("u_rep", 0.0)), float(d.get("sgn", 1.0))
            c.j = int(d.get("j", 0))
            for k, v in enumerate(d.get("km", [])):
                c.km[k] = int(v)
            for k, v in enumerate(d.get("kp", [])):
                c.kp[k] = int(v)
            m = np.ascontiguousarray(d.get("mask", np.zeros(self.dim)), dtype=np.uint8)
            u = np.ascontiguousarray(d.get("U", np.zeros(self.dim)), dtype=np.float64)
            if m.shape != (self.dim,) or u.shape != (self.dim,):
                raise ValueError("mask and U hold one value per coordinate")
            keep += [m, u]
            c.mask = _ptr(m, C.c_uint8)
            c.U = _ptr(u, C.c_double)
        tr, c_tr, drc = self._trace()
        s = self._c()
        rc = self._lib().oracle_step_scripted(C.byref(s), int(t), _ptr(X, C.c_double),
                                              _ptr(F, C.c_double), recs, C.byref(c_tr))
        if rc != 0:
            raise ValueError(f"oracle_step_scripted rejected t={t}")
        tr.dr_count = int(drc[0])
        tr.accepted = tr.accepted.astype(bool)
        return X, F, tr

    def run(self, X, F, t0: int, iters: int):
        X = np.array(X, dtype=np.float64, order="C")
        F = np.array(F, dtype=np.float64)
        s = self._c()
        t = self._lib().oracle_run(C.byref(s), int(t0), int(iters), _ptr(X, C.c_double),
                             _ptr(F, C.c_double))
        return X, F, int(t)

    def solve(self):
        """Init + all iterations; returns (x_best, f_best, X, F)."""
        X, F = self.init()
        X, F, _ = self.run(X, F, 0, self.max_iter)
        b = best(F)
        return X[b].copy(), float(F[b]), X, F

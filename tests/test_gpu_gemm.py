"""The GEMM form of the step (rotated objectives of large dimension, and the
BF16 form).  The binary32 GEMM form follows the oracle within the binary32
tolerances; the BF16 form -- a BF16 estimate, then a binary32 re-score of
every candidate the estimate cannot settle under its bound and of every
acceptance -- must store exactly what the binary32 form stores, iteration
after iteration; the elite's fitness is re-scored in binary64 and equals
the oracle's objective of the returned position."""
import numpy as np
import pytest

import gen
import oracle as O
from gpu_common import compare_step, make_pair, need_gpu, random_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["rastrigin", "ackley", "sphere"])
def test_fp32_gemm_form_step_parity(kind):
    apo = need_gpu()
    print(f"[gemm] fp32 D600 {kind}", flush=True)
    g, p = make_pair(apo, dim=600, pop=70, kind=kind, rotated=True, precision="fp32",
                     max_iter=20, seed=4, pf_max=0.3)
    with g:
        for sseed in (3, 4):
            X, F = random_state(p, sseed, "fp32")
            compare_step(g, p, 5, X, F, "fp32")


def _pair(apo, dim, pop, kind, T, seed):
    w = gen.rotated_rastrigin_large(seed=seed, pop=pop, dim=dim, max_iter=T)
    kw = dict(np_pairs=1, pf_max=0.1, seed=seed, max_iter=T, kind=kind, shift=w.shift, rot=w.rot)
    a = apo.APO(dim, w.lb, w.ub, pop, precision="fp32", **kw)
    b = apo.APO(dim, w.lb, w.ub, pop, precision="bf16", **kw)
    return w, a, b


@pytest.mark.parametrize("kind", ["ackley", "rastrigin"])
def test_bf16_form_equals_fp32_form(kind):
    apo = need_gpu()
    print(f"[gemm] bf16 vs fp32 D520 {kind}", flush=True)
    w, a, b = _pair(apo, 520, 200, kind, 30, 6)
    with a, b:
        for _ in range(3):
            a.run(10)
            b.run(10)
            Xa, Fa, ta = a.get_state()
            Xb, Fb, tb = b.get_state()
            assert ta == tb
            assert np.array_equal(Xa, Xb) and np.array_equal(Fa, Fb)
        x, f, _ = b.best()
        p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind=kind, shift=w.shift, rot=w.rot)
        fo = p.objective(x)
        assert abs(f - fo) <= 1e-10 * max(1.0, abs(fo))


def test_bf16_form_small_dimension_and_elite():
    """BF16 is a precision, not a size: at D 64 it runs the GEMM form too
    (a binary32 handle of that size runs the tiled form, so the comparison
    is with the oracle)."""
    apo = need_gpu()
    print("[gemm] bf16 D64", flush=True)
    g, p = make_pair(apo, dim=64, pop=96, kind="ackley", rotated=True, precision="bf16",
                     max_iter=10, seed=9)
    with g:
        g.run(10)
        X, F, t = g.get_state()
        assert t == 10 and np.all(np.isfinite(F))
        assert np.all(X >= p.lb) and np.all(X <= p.ub)
        for i in range(0, 96, 17):   # stored fitness = binary32 value of the stored row
            fo = p.objective(X[i])
            assert abs(F[i] - fo) <= 1e-4 * (abs(fo) + 1.0), i
        x, f, _ = g.best()
        assert abs(f - p.objective(x)) <= 1e-10 * max(1.0, abs(f))


def test_precision_pipeline_full_size():
    """The precision configuration's shape: ps 8192, D 1000, shifted-rotated
    Ackley.  Two iterations of the BF16 and binary32 forms store the same
    rows and fitness; the elite re-scored in binary64 matches the oracle."""
    apo = need_gpu()
    print("[gemm] ps8192 D1000 ackley, 2 iterations", flush=True)
    w, a, b = _pair(apo, 1000, 8192, "ackley", 2000, 1)
    with a, b:
        a.run(2)
        b.run(2)
        Xa, Fa, _ = a.get_state()
        Xb, Fb, _ = b.get_state()
        assert np.array_equal(Fa, Fb)
        assert np.array_equal(Xa, Xb)
        x, f, _ = b.best()
        p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind="ackley", shift=w.shift,
                      rot=w.rot)
        assert abs(f - p.objective(x)) <= 1e-10 * max(1.0, abs(f))


def test_bf16_settled_rejections_keep_parents():
    """Sphere at D 520: the bound is a fixed fraction of the fitness, so
    candidates far worse than their parents are rejected on the BF16
    estimate alone (the parent row and fitness carried over without a
    binary32 re-score).  The run still equals the binary32 form's."""
    apo = need_gpu()
    print("[gemm] bf16 vs fp32 D520 sphere, settled rejections", flush=True)
    w, a, b = _pair(apo, 520, 256, "sphere", 40, 11)
    with a, b:
        for _ in range(4):
            a.run(10)
            b.run(10)
            Xa, Fa, ta = a.get_state()
            Xb, Fb, tb = b.get_state()
            assert ta == tb
            assert np.array_equal(Xa, Xb) and np.array_equal(Fa, Fb)
        rescored, estimated = b.precision_stats()
        print(f"[gemm] re-scored {rescored} of {estimated}", flush=True)
        assert estimated == 40 * 256
        assert 0 < rescored < estimated


@pytest.mark.parametrize("dim,pop", [(1, 2), (17, 3), (129, 300)])
def test_bf16_form_ragged_shapes(dim, pop):
    """The BF16 form at ragged sizes (K and N padding, a partial row block,
    more than one row block): finite fitness, rows in bounds, the stored
    fitness equal to the objective of the stored row within binary32
    rounding, and the elite re-scored in binary64."""
    apo = need_gpu()
    print(f"[gemm] bf16 ragged D{dim} ps{pop}", flush=True)
    g, p = make_pair(apo, dim=dim, pop=pop, kind="rastrigin", rotated=True, precision="bf16",
                     max_iter=6, seed=5, pf_max=0.5)
    with g:
        g.run(6)
        X, F, t = g.get_state()
        assert t == 6 and np.all(np.isfinite(F))
        assert np.all(X >= p.lb) and np.all(X <= p.ub)
        for i in range(0, pop, max(1, pop // 7)):
            fo = p.objective(X[i])
            assert abs(F[i] - fo) <= 1e-4 * (abs(fo) + 1.0), i
        x, f, _ = g.best()
        assert abs(f - p.objective(x)) <= 1e-10 * max(1.0, abs(f))

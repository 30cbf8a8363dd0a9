"""Pins for the oracle's objectives and its sort order.

Each objective is pinned to something other than the oracle's own formula:
the worked example's printed Sphere values (Section 4.1, Step 1), closed
forms at special points, library routines (scipy's Rosenbrock and entropy,
numpy's stable argsort), invariants of orthogonal rotations, and brute force
against an exact dynamic programme for the thresholding criteria.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import optimize, stats

import gen
import oracle as O


def prob(kind, dim, shift=None, rot=None, hist=None, lb=-100.0, ub=100.0):
    return O.Problem(dim=dim, pop=2, lb=lb, ub=ub, kind=kind, shift=shift, rot=rot, hist=hist)


def test_sphere_matches_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    p = prob("sphere", 3, lb=g["lb"], ub=g["ub"])
    for x, f in zip(g["step1_population"], g["step1_fitness_printed"]):
        assert abs(p.objective(x) - f) <= 0.5 * 10 ** -g["printed_decimals"] + 1e-12


@pytest.mark.parametrize("dim", [1, 2, 10, 100])
def test_rastrigin_zero_at_shift_and_integer_lattice(dim):
    o = gen.shift_vector(dim, seed=3)
    p = prob("rastrigin", dim, shift=o)
    assert p.objective(o) == 0.0
    # unshifted: at an integer point n the cosine term vanishes and f = |n|^2
    q = prob("rastrigin", dim)
    n = np.random.default_rng(dim).integers(-5, 6, size=dim).astype(float)
    assert abs(q.objective(n) - float(n @ n)) <= 1e-10 * max(1.0, float(n @ n))
    # and at half-integers cos(2 pi z) = -1: f = |z|^2 + 20 dim
    h = n + 0.5
    assert abs(q.objective(h) - (float(h @ h) + 20.0 * dim)) <= 1e-9 * float(h @ h + 20 * dim)


@pytest.mark.parametrize("dim", [2, 3, 10, 50])
def test_rosenbrock_vs_scipy_with_permutation_rotation(dim):
    rng = np.random.default_rng(dim)
    o = gen.shift_vector(dim, seed=5)
    sigma = rng.permutation(dim)
    M = np.zeros((dim, dim))
    M[np.arange(dim), sigma] = 1.0            # (M v)_i = v_sigma(i)
    p = prob("rosenbrock", dim, shift=o, rot=M)
    for _ in range(5):
        x = rng.uniform(-100, 100, size=dim)
        z = (x - o)[sigma]
        want = optimize.rosen(z + 1.0)
        assert abs(p.objective(x) - want) <= 1e-12 * max(1.0, abs(want))
    assert p.objective(o) == 0.0
    if dim > 2:
        # the transposed matrix is a different permutation and gives a different value
        pt = prob("rosenbrock", dim, shift=o, rot=M.T.copy())
        x = rng.uniform(-100, 100, size=dim)
        if not np.array_equal(sigma, np.argsort(sigma)):
            assert pt.objective(x) != p.objective(x)


@pytest.mark.parametrize("dim", [1, 10, 100])
def test_ackley_closed_forms(dim):
    o = gen.shift_vector(dim, seed=7)
    p = prob("ackley", dim, shift=o)
    assert abs(p.objective(o)) <= 1e-14
    q = prob("ackley", dim)
    for c in (1, 2, -3, 7):
        x = np.full(dim, float(c))
        want = 20.0 * (1.0 - math.exp(-0.2 * abs(c)))
        assert abs(q.objective(x) - want) <= 1e-12


@pytest.mark.parametrize("dim", [2, 10, 100])
def test_rotation_generator_and_orthogonal_invariance(dim):
    M = gen.rotation_matrix(dim, seed=11)
    assert np.abs(M.T @ M - np.eye(dim)).max() <= 1e-13
    o = gen.shift_vector(dim, seed=11)
    rot = prob("sphere", dim, shift=o, rot=M)
    plain = prob("sphere", dim, shift=o)
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.uniform(-100, 100, size=dim)
        a, b = rot.objective(x), plain.objective(x)
        assert abs(a - b) <= 1e-11 * b
    # rotated Rastrigin is still exactly 0 at the shift point
    assert prob("rastrigin", dim, shift=o, rot=M).objective(o) == 0.0


def test_sort_order_matches_numpy_stable_argsort():
    vals = [-1.0, -0.0, 0.0, 1.0, float("nan"), float("inf")]
    for n in range(1, 6):
        for combo in itertools.product(vals, repeat=n):
            F = np.array(combo)
            assert np.array_equal(O.rank_order(F), np.argsort(F, kind="stable")), combo
    rng = np.random.default_rng(2)
    F = rng.integers(0, 20, size=4096).astype(float)      # many ties
    assert np.array_equal(O.rank_order(F), np.argsort(F, kind="stable"))
    assert O.best(F) == int(np.argsort(F, kind="stable")[0])


# --------------------------- thresholding ---------------------------------

def _class_entropy(h, a, b):
    seg = np.asarray(h[a:b], dtype=float)
    return 0.0 if seg.sum() == 0 else float(stats.entropy(seg))


def _kapur_dp(h, k):
    """Exact optimum of sum_c H(class c) over 0 <= b1 <= ... <= bk <= 256,
    by dynamic programming over the last boundary (H is additive over
    consecutive classes)."""
    L = 257
    best = np.full((k + 2, L), -np.inf)
    best[0, 0] = 0.0
    for c in range(1, k + 2):
        for b in range(L):
            cand = [best[c - 1, a] + _class_entropy(h, a, b) for a in range(b + 1)
                    if best[c - 1, a] > -np.inf]
            best[c, b] = max(cand) if cand else -np.inf
    return best[k + 1, 256]


def test_kapur_uniform_histogram_closed_form():
    h = np.full(256, 10, dtype=np.uint64)
    p = prob("kapur", 1, hist=h, lb=0.0, ub=255.0)
    assert abs(p.objective([128.0]) - (-2.0 * math.log(128.0))) <= 1e-12
    p3 = prob("kapur", 3, hist=h, lb=0.0, ub=255.0)
    assert abs(p3.objective([64.0, 192.0, 128.0]) - (-4.0 * math.log(64.0))) <= 1e-12
    # rounding is half to even: 127.5 -> 128, 128.5 -> 128
    assert p.objective([127.5]) == p.objective([128.0]) == p.objective([128.5])


def test_kapur_matches_scipy_entropy_per_class():
    rng = np.random.default_rng(4)
    h = rng.integers(0, 50, size=256).astype(np.uint64)
    h[rng.integers(0, 256, size=40)] = 0
    for k in (1, 2, 4, 8, 16):
        p = prob("kapur", k, hist=h, lb=0.0, ub=255.0)
        for _ in range(10):
            x = rng.uniform(0, 255, size=k)
            t = sorted(int(np.rint(v)) for v in x)
            bounds = [0] + t + [256]
            want = -sum(_class_entropy(h, bounds[c], bounds[c + 1]) for c in range(k + 1))
            assert abs(p.objective(x) - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("L,k", [(8, 1), (8, 2), (8, 3), (16, 1), (16, 2), (16, 3), (32, 1), (32, 2)])
def test_kapur_brute_force_equals_dp(L, k):
    rng = np.random.default_rng(L * 10 + k)
    h = np.zeros(256, dtype=np.uint64)
    h[:L] = rng.integers(0, 20, size=L)
    h[rng.integers(0, L)] += 5
    p = prob("kapur", k, hist=h, lb=0.0, ub=255.0)
    best = min(p.objective(np.array(t, dtype=float))
               for t in itertools.combinations_with_replacement(range(L + 1), k))
    assert abs(best - (-_kapur_dp(h, k))) <= 1e-12


def test_otsu_two_class_identity():
    rng = np.random.default_rng(9)
    h = rng.integers(0, 100, size=256).astype(np.uint64)
    p = prob("otsu", 1, hist=h, lb=0.0, ub=255.0)
    pr = h / h.sum()
    g = np.arange(256)
    for t in (1, 50, 128, 200, 255):
        w0, w1 = pr[:t].sum(), pr[t:].sum()
        m0 = (g[:t] * pr[:t]).sum() / w0
        m1 = (g[t:] * pr[t:]).sum() / w1
        want = -(w0 * w1 * (m0 - m1) ** 2)        # textbook two-class form
        assert abs(p.objective([float(t)]) - want) <= 1e-10 * abs(want)

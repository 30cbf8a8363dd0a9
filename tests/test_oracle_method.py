"""Pins for the oracle's APO step (Section 3, Algorithm 1, Section 4.1).

The worked example (Section 4.1) fixes the sort, the size of Dr, the sizes
of the foraging masks, the bound clamp, the evaluated candidates and the
strict greedy selection.  Closed-form limits of Eqs. (4), (12) and (13) and
invariants of Eqs. (1), (2), (6) and (8) (independence from X, clone
populations, translation and scale equivariance, the sign of the neighbour
difference) pin the update formulas; determinism and resume pin the absence
of hidden state.
"""
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle as O

DORM, REPRO, AUTO, HETERO = 0, 1, 2, 3


@pytest.fixture(scope="module")
def example(golden_dir):
    return json.load(open(os.path.join(golden_dir, "worked_example.json")))


def example_problem(g, seed=1, max_iter=100):
    return O.Problem(dim=g["dim"], pop=g["pop"], lb=g["lb"], ub=g["ub"], pf_max=g["pf_max"],
                     kind="sphere", seed=seed, max_iter=max_iter)


def test_example_step2_sort(example):
    X = np.array(example["step1_population"])
    p = example_problem(example)
    F = np.array([p.objective(x) for x in X])
    perm = O.rank_order(F)
    assert np.allclose(X[perm], example["step2_sorted_population"])
    assert np.allclose(np.round(F[perm], 2), example["step2_sorted_fitness_printed"])


def test_example_step3_and_step5_counts(example):
    """|Dr| = ceil(ps pf) = 1 (Step 3); a foraging protozoan of rank i changes
    at most ceil(dim i / ps) coordinates: 1 for rank 1 (1.2 -> 1.77) and all
    3 for ranks 3 and 4 (Step 5)."""
    X = np.array(example["step1_population"])
    printed_changes = [int(np.sum(np.array(a) != np.array(b)))
                       for a, b in zip(example["step2_sorted_population"],
                                       example["step5_candidates_by_rank"])]
    assert printed_changes == [1, 2, 3, 3]
    mf = [math.ceil(3 * i / 4) for i in range(1, 5)]
    assert [printed_changes[0], printed_changes[2], printed_changes[3]] == [mf[0], mf[2], mf[3]]
    for seed in range(1, 200):
        p = example_problem(example, seed=seed)
        F = np.array([p.objective(x) for x in X])
        _, _, tr = p.step(1, X, F)
        assert tr.dr_count == example["step3_dr_size"]
        assert int(np.sum((tr.op == DORM) | (tr.op == REPRO))) == 1
        for r, idx in enumerate(tr.perm):
            changed = int(np.sum(tr.Y[idx] != X[idx]))
            if tr.op[idx] in (AUTO, HETERO):
                assert tr.mcount[idx] == mf[r]
                assert changed <= mf[r]
            elif tr.op[idx] == REPRO:
                assert 1 <= tr.mcount[idx] <= 3 and changed <= tr.mcount[idx]


def test_example_step6_clamp_evaluate_select(example):
    X = np.array(example["step2_sorted_population"])
    p = example_problem(example)
    F = np.array([p.objective(x) for x in X])
    Xn, Fn, Yc, Fy, acc = p.finish(X, F, np.array(example["step5_candidates_by_rank"]))
    assert np.allclose(Yc, example["step6_clamped_by_rank"], atol=0)
    tol = 0.5 * 10 ** -example["printed_decimals"]
    # the printed candidates are themselves rounded; allow their 0.005 slack
    for f, want in zip(Fy, example["step6_candidate_fitness_printed"]):
        assert abs(f - want) <= tol + 0.01
    assert acc.tolist() == [False, False, True, True]
    assert np.allclose(Xn, example["step6_next_population_by_rank"], atol=0)


def _state(kind="sphere", dim=6, pop=12, seed=3, T=50, **kw):
    lb, ub = -10.0, 10.0
    p = O.Problem(dim=dim, pop=pop, lb=lb, ub=ub, kind=kind, seed=seed, max_iter=T, **kw)
    X = gen.random_state(pop, dim, p.lb, p.ub, seed)
    F = np.array([p.objective(x) for x in X])
    return p, X, F


def test_bounds_fixed_population_and_monotone_best():
    for kind in ("sphere", "rastrigin", "ackley", "rosenbrock"):
        p, X, F = _state(kind, pf_max=0.5, shift=gen.shift_vector(6, 2, -8, 8))
        bests = [F.min()]
        for t in range(1, p.max_iter + 1):
            X, F, _ = p.step(t, X, F, trace=False)
            assert X.shape == (12, 6)
            assert np.all(X >= p.lb) and np.all(X <= p.ub)
            assert np.allclose(F, [p.objective(x) for x in X], rtol=0, atol=0)
            bests.append(F.min())
        assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
        assert bests[-1] < bests[0]


def test_last_iteration_leaves_foraging_rows_unchanged():
    """At t = T the factor of Eq. (4) and p_ah of Eq. (12) are 0: every
    foraging protozoan is a heterotroph whose candidate equals its row, and
    the strict selection keeps the row."""
    p, X, F = _state(pf_max=0.3)
    X1, F1, tr = p.step(p.max_iter, X, F)
    forage = (tr.op == AUTO) | (tr.op == HETERO)
    assert np.all(tr.op[forage] == HETERO)
    assert np.array_equal(tr.Y[forage], X[forage])
    assert not np.any(tr.accepted[forage])
    assert np.array_equal(X1[forage], X[forage])


def test_first_iterations_are_mostly_autotrophs():
    p, X, F = _state(pop=64, T=1000, pf_max=0.0)
    _, _, tr = p.step(1, X, F)
    assert tr.dr_count == 0 and np.all(tr.op >= AUTO)
    assert np.mean(tr.op == AUTO) > 0.9              # p_ah(1) ~ 1


def test_dormancy_probability_follows_eq13():
    """Eq. (13) as printed: p_dr = (1 - cos((1 - i/ps) pi)) / 2 is ~1 for the
    best rank and exactly 0 for the worst, so in Dr the best rank goes
    dormant and the worst always reproduces."""
    p, X, F = _state(pop=16, pf_max=1.0, T=10)
    best_n = best_dorm = worst_n = worst_dorm = 0
    for seed in range(1, 400):
        p.seed = seed
        _, _, tr = p.step(3, X, F)
        b, w = tr.op[tr.perm[0]], tr.op[tr.perm[-1]]
        if b in (DORM, REPRO):
            best_n += 1
            best_dorm += b == DORM
        if w in (DORM, REPRO):
            worst_n += 1
            worst_dorm += w == DORM
    assert best_n > 20 and worst_n > 20
    assert worst_dorm == 0
    assert best_dorm >= best_n - 1


def test_dormancy_variant_mirrors_eq13():
    """The opposite sign in Eq. (13) (a variant): p_dr = (1 + cos((1 - i/ps)
    pi)) / 2 is exactly 1 for the worst rank and ~0 for the best, so in Dr
    the worst rank always goes dormant and the best almost never does; the
    variant and the printed form add up to 1 at every rank."""
    p, X, F = _state(pop=16, pf_max=1.0, T=10)
    p.pdr_plus = True
    best_n = best_dorm = worst_n = worst_dorm = 0
    for seed in range(1, 400):
        p.seed = seed
        _, _, tr = p.step(3, X, F)
        b, w = tr.op[tr.perm[0]], tr.op[tr.perm[-1]]
        if b in (DORM, REPRO):
            best_n += 1
            best_dorm += b == DORM
        if w in (DORM, REPRO):
            worst_n += 1
            worst_dorm += w == DORM
    assert best_n > 20 and worst_n > 20
    assert worst_dorm == worst_n
    assert best_dorm <= 2
    # same draws, opposite decisions wherever u_op lies between the two forms
    p.seed = 5
    p.pdr_plus = False
    _, _, a = p.step(3, X, F)
    p.pdr_plus = True
    _, _, b = p.step(3, X, F)
    dr = np.isin(a.op, (DORM, REPRO))
    assert np.array_equal(dr, np.isin(b.op, (DORM, REPRO)))   # Dr itself is unchanged


def test_dormancy_ignores_the_row_and_reproduction_keeps_unmasked_dims():
    p, X, F = _state(pop=16, pf_max=1.0)
    X2 = gen.random_state(16, 6, p.lb, p.ub, seed=99)
    _, _, tr1 = p.step(2, X, F)
    _, _, tr2 = p.step(2, X2, F)                     # same F: same sort and draws
    d = tr1.op == DORM
    assert d.any()
    assert np.array_equal(tr1.Y[d], tr2.Y[d])        # Eq. (1) does not read X_i
    rep = np.where(tr1.op == REPRO)[0]
    assert rep.size
    for i in rep:
        assert np.sum(tr1.Y[i] != X[i]) <= tr1.mcount[i]


def test_autotroph_clones_stay_put():
    """With every row equal, X_j - X_i and X_k- - X_k+ vanish in Eq. (6)."""
    p, X, F = _state(pop=16, pf_max=0.0, T=100)
    Xc = np.tile(X[0], (16, 1))
    Fc = np.full(16, F[0])
    _, _, tr = p.step(5, Xc, Fc)
    a = tr.op == AUTO
    assert a.any()
    assert np.array_equal(tr.Y[a], Xc[a])


def test_autotroph_translation_equivariance():
    """Eq. (6) is affine in the rows with coefficients that sum to one, so
    translating the population (and the bounds) translates the candidates."""
    p, X, F = _state(pop=16, pf_max=0.0, T=100)
    shift = 4.0
    q = O.Problem(dim=p.dim, pop=p.pop, lb=p.lb + shift, ub=p.ub + shift, kind="sphere",
                  seed=p.seed, max_iter=p.max_iter, pf_max=0.0)
    _, _, t1 = p.step(5, X, F)
    _, _, t2 = q.step(5, X + shift, F)               # same F keeps sort and draws
    a = t1.op == AUTO
    assert a.any()
    inside = np.all((t1.Y > p.lb) & (t1.Y < p.ub), axis=1) & a
    assert np.allclose(t2.Y[inside], t1.Y[inside] + shift, rtol=0, atol=1e-12)


def test_scale_equivariance_of_every_operation():
    """Every candidate is homogeneous of degree one in (X, X_min, X_max):
    scaling both by 2 (exact in binary) scales the candidates by 2."""
    p, X, F = _state(pop=24, pf_max=0.6, T=40)
    q = O.Problem(dim=p.dim, pop=p.pop, lb=2 * p.lb, ub=2 * p.ub, kind="sphere",
                  seed=p.seed, max_iter=p.max_iter, pf_max=0.6)
    ops = set()
    for t in (1, 7, 20, 30, 38):
        _, _, t1 = p.step(t, X, F)
        _, _, t2 = q.step(t, 2 * X, F)
        assert np.array_equal(t2.Y, 2 * t1.Y)
        ops |= set(t1.op.tolist())
    assert ops == {DORM, REPRO, AUTO, HETERO}


def test_heterotroph_moves_toward_the_better_neighbour():
    """Eq. (8): for X_i = 0 the X_near term vanishes and the candidate is
    f * w * (X_{i-1} - X_{i+1}) on its mask: it points from the worse
    neighbour toward the better one."""
    pop, dim = 9, 5
    p = O.Problem(dim=dim, pop=pop, lb=-10.0, ub=10.0, kind="sphere", pf_max=0.0, max_iter=4)
    F = np.arange(pop, dtype=float) + 1.0            # id == rank
    X = np.zeros((pop, dim))
    X[:4] = 1.0                                      # better ranks at +1
    X[5:] = -1.0                                     # worse ranks at -1
    seen = 0
    for seed in range(1, 80):
        p.seed = seed
        _, _, tr = p.step(3, X, F)
        if tr.op[4] != HETERO:
            continue
        seen += 1
        moved = tr.Y[4][tr.Y[4] != 0.0]
        assert moved.size == tr.mcount[4] and np.all(moved > 0.0)
        assert tr.nb[4].tolist() == [-1, 3, 5]
    assert seen > 5


def test_autotroph_neighbour_ranks():
    """k- is a strictly better rank (itself for the best), k+ a strictly
    worse one (itself for the worst), j any rank; the draws are uniform."""
    pop = 10
    p, X, F = _state(pop=pop, pf_max=0.0, T=1000)
    counts_j = np.zeros(pop)
    counts_km = np.zeros((pop, pop))
    for seed in range(1, 150):
        p.seed = seed
        _, _, tr = p.step(2, X, F)
        for r, idx in enumerate(tr.perm):
            if tr.op[idx] != AUTO:
                continue
            j, km, kp = tr.nb[idx]
            assert 0 <= j < pop
            assert (km < r) if r > 0 else (km == r)
            assert (kp > r) if r < pop - 1 else (kp == r)
            counts_j[j] += 1
            counts_km[r, km] += 1
    from scipy import stats
    assert stats.chisquare(counts_j).pvalue > 1e-4
    row = counts_km[pop - 1, : pop - 1]
    assert stats.chisquare(row).pvalue > 1e-4


def test_deterministic_and_resumable():
    w = gen.shifted_rastrigin_small(seed=4)
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind=w.kind, shift=w.shift,
                  seed=w.seed, max_iter=w.max_iter)
    X0, F0 = p.init()
    assert np.all(X0 >= p.lb) and np.all(X0 <= p.ub)
    Xa, Fa, ta = p.run(X0, F0, 0, w.max_iter)
    Xb, Fb, tb = p.run(X0, F0, 0, w.max_iter)
    assert ta == tb == w.max_iter
    assert np.array_equal(Xa, Xb) and np.array_equal(Fa, Fb)
    Xm, Fm, tm = p.run(X0, F0, 0, 77)
    Xc, Fc, tc = p.run(Xm, Fm, tm, w.max_iter)
    assert tc == w.max_iter and np.array_equal(Xa, Xc) and np.array_equal(Fa, Fc)
    # a different run id changes the stream
    q = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind=w.kind, shift=w.shift,
                  seed=w.seed, max_iter=w.max_iter, run_id=1)
    Xq, Fq, _ = q.run(X0, F0, 0, 5)
    Xp, Fp, _ = p.run(X0, F0, 0, 5)
    assert not np.array_equal(Xq, Xp)


def test_small_rastrigin_run_improves():
    w = gen.shifted_rastrigin_small(seed=1)
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind=w.kind, shift=w.shift,
                  seed=w.seed, max_iter=w.max_iter)
    X0, F0 = p.init()
    xb, fb, X, F = p.solve()
    assert fb < 0.05 * F0.min()
    assert fb == F.min() and np.array_equal(xb, X[O.best(F)])


def test_histogram_matches_bincount():
    img = gen.blob_image(96, 80, seed=3)
    assert np.array_equal(O.histogram_u8(img), np.bincount(img.reshape(-1), minlength=256))
    for const in (0, 255, 17):
        im = np.full((33, 7), const, np.uint8)
        h = O.histogram_u8(im)
        assert h[const] == im.size and h.sum() == im.size


def test_rank_order_is_reentrant_across_host_threads():
    """The sort is called from several host threads at once (seeds of the
    distribution tests run in parallel): each call keeps its own array."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(7)
    arrays = [rng.integers(0, 50, size=200_000).astype(np.float64) for _ in range(8)]
    want = [np.argsort(F, kind="stable") for F in arrays]
    with ThreadPoolExecutor(max_workers=8) as ex:
        for _ in range(3):
            got = list(ex.map(O.rank_order, arrays))
            for g, w in zip(got, want):
                assert np.array_equal(g, w)

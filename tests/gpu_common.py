"""Helpers shared by the GPU tests: building matching GPU/oracle problems,
injecting one state into both, and the tolerances the comparisons use.

Tolerances (derived from the arithmetic; eps = unit roundoff of the
handle's precision):
  * integer work -- rank permutation, operation codes, Dr, masks (seen
    through which coordinates move), thresholds -- is compared exactly;
  * binary64 candidates follow the oracle's expression order; only the
    weights of Eqs. (7)/(10) go through exp, whose last-bit difference
    between libraries scales with the moved distance, so
    |dY| <= 64 eps64 (|X_i| + |Y - X_i| + 1);
  * binary32 candidates: |dY| <= 1e-5 (|X_i| + |Y - X_i|) + 1e-6;
  * fitness: |dF| <= c * (sum_d |g_d| + 10 D) with c = 64 D eps64 in
    binary64 and 1e-5 in binary32 (forward error of a D-term sum of
    terms of size |g_d|, plus the cosine terms); rotated objectives add
    the error of z = M (y - o): sum_d |g'(z_d)| * D eps sum_j |M_dj| |v_j|;
  * selection decisions must agree except where the oracle's candidate
    fitness is within that tolerance of the old fitness (a near tie).
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle as O

EPS64 = np.finfo(np.float64).eps
OP_NAMES = {0: "dormancy", 1: "reproduction", 2: "autotroph", 3: "heterotroph"}


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_14982_amd as apo
    return apo


def make_pair(apo, *, dim, pop, kind="rastrigin", precision="fp64", rotated=False, np_pairs=1,
              pf_max=0.1, seed=1, max_iter=100, lb=-100.0, ub=100.0, shift=True, hist=None,
              trace=True, run_id=0, pdr_plus=False):
    dt = np.float32 if precision in ("fp32", "bf16") else np.float64
    lbv = np.broadcast_to(np.asarray(lb, np.float64), (dim,)).astype(dt).astype(np.float64)
    ubv = np.broadcast_to(np.asarray(ub, np.float64), (dim,)).astype(dt).astype(np.float64)
    o = None
    M = None
    if kind not in ("kapur", "otsu"):
        if shift:
            o = gen.shift_vector(dim, seed, -0.8 * float(np.max(np.abs(ubv))),
                                 0.8 * float(np.max(np.abs(ubv))), dtype=dt)
        if rotated:
            M = gen.rotation_matrix(dim, seed, dtype=dt)
    g = apo.APO(dim, lbv, ubv, pop, np_pairs=np_pairs, pf_max=pf_max, seed=seed, max_iter=max_iter,
                precision=precision, kind=kind, shift=o, rot=M, hist=hist, trace=trace,
                run_id=run_id, pdr_plus=pdr_plus)
    p = O.Problem(dim=dim, pop=pop, lb=lbv, ub=ubv, np_pairs=np_pairs, max_iter=max_iter,
                  pf_max=pf_max, seed=seed, run_id=run_id, kind=kind, shift=o, rot=M, hist=hist,
                  pdr_plus=pdr_plus)
    return g, p


def random_state(p, seed, precision):
    dt = np.float32 if precision == "fp32" else np.float64
    X = gen.random_state(p.pop, p.dim, p.lb, p.ub, seed, dtype=dt)
    F = np.array([p.objective(x) for x in X]).astype(dt).astype(np.float64)
    return X, F


def fitness_terms(p, y):
    """(sum_d |g_d| + 10 D, rotation error scale) of a candidate, from the
    oracle's definitions of the objectives (used only to size tolerances)."""
    D = p.dim
    v = y - (p.shift if p.shift is not None else 0.0)
    z = p.rot @ v if p.rot is not None else v
    if p.kind == "rastrigin":
        g = np.abs(z * z - 10 * np.cos(2 * np.pi * z) + 10)
        gp = 2 * np.abs(z) + 20 * np.pi
    elif p.kind == "sphere":
        g = z * z
        gp = 2 * np.abs(z)
    elif p.kind == "rosenbrock":
        a = z[:-1] + 1
        b = z[1:] + 1
        g = np.concatenate([100 * (b - a * a) ** 2 + (a - 1) ** 2, [0.0]])
        gp = np.concatenate([400 * np.abs(a) * np.abs(b - a * a) + 2 * np.abs(a - 1), [0.0]]) + \
            np.concatenate([[0.0], 200 * np.abs(b - a * a)])
    elif p.kind == "ackley":
        g = np.full(D, (20 + np.e) / D) + np.abs(z) * 0
        gp = np.full(D, 2 * np.pi + 4.0)
    else:
        return 10.0, 0.0
    scale = g.sum() + 10 * D
    rot_err = 0.0
    if p.rot is not None:
        dz = D * np.abs(p.rot) @ np.abs(v)
        rot_err = float((gp * dz).sum())
    return float(scale), rot_err


def f_tolerance(p, y, precision):
    scale, rot_err = fitness_terms(p, y)
    if p.kind in ("kapur", "otsu"):
        # class sums taken as differences of prefix tables (binary64) and,
        # for a binary32 handle, the final rounding of F to binary32
        f = abs(p.objective(y))
        return (1e-9 if precision == "fp64" else 1e-6) * (f + 1.0)
    if precision == "fp64":
        return 64 * p.dim * EPS64 * scale + 4 * EPS64 * rot_err + 1e-300
    return 1e-5 * scale + 1e-6 * rot_err + 1e-6


def y_tolerance(x, y, precision, mag=0.0):
    """Candidate tolerance: relative to the row and the move, plus a term in
    the largest operand the coordinate is computed from (mag): rounding in
    Eqs. (1), (2), (6)-(10) is relative to the bounds and the neighbour rows,
    which can be far larger than the result."""
    if precision == "fp64":
        return 64 * EPS64 * (np.abs(x) + np.abs(y - x) + 1.0 + mag)
    return 1e-5 * (np.abs(x) + np.abs(y - x)) + 1e-6 * mag + 1e-6


def operand_magnitude(p, X, tr):
    """Per candidate coordinate, the largest operand magnitude its formula
    reads: the bounds for dormancy and reproduction (Eqs. (1), (2)), the own
    row and the neighbour rows for the foraging modes (Eqs. (6)-(10))."""
    bnd = np.maximum(np.abs(np.broadcast_to(np.asarray(p.lb, float), (p.dim,))),
                     np.abs(np.broadcast_to(np.asarray(p.ub, float), (p.dim,))))
    mag = np.abs(X).astype(np.float64)
    forage = tr.op >= 2
    for c in range(tr.nb.shape[1]):
        ids = tr.nb[:, c]
        ok = forage & (ids >= 0)
        mag[ok] = np.maximum(mag[ok], np.abs(X[ids[ok]]))
    mag[~forage] = np.maximum(mag[~forage], bnd)
    return mag


def compare_step(g, p, t, X, F, precision, exact_dr=True, bf16=False):
    """Inject (X, F) at iteration t-1 into both sides, run one step and
    compare everything the step produces."""
    g.set_state(X, F, t - 1)
    assert g.step()
    return check_step(g, p, t, X, F, precision, bf16=bf16)


def check_step(g, p, t, X, F, precision, bf16=False):
    """Compare the step g has just taken from (X, F) at iteration t-1 with
    the oracle's iteration t from the same state.  With bf16, fitness values
    the BF16 estimate settled (rejections it proved) are not binary32
    values: those rows are only required to be rejected by the oracle too
    (or to be near ties), accepted rows must carry the binary32 fitness."""
    Yg, Fyg, opg, permg = g.get_trace()
    Xg, Fg, tg = g.get_state()
    Xo, Fo, tr = p.step(t, X, F)
    assert tg == t
    # integer work: exact
    assert np.array_equal(permg, tr.perm), "rank permutation differs"
    assert np.array_equal(opg, tr.op), "operation choice differs"
    # candidates
    if p.kind in ("kapur", "otsu"):
        # the thresholds are what the objective sees: compare them exactly
        # except where the candidate sits within tolerance of a half level
        tol = y_tolerance(X, tr.Y, precision)
        assert np.all(np.abs(Yg - tr.Y) <= tol), "threshold candidates differ"
        frac = np.abs(tr.Y - np.floor(tr.Y) - 0.5)
        clear = frac > 1e-4
        assert np.array_equal(np.rint(Yg)[clear], np.rint(tr.Y)[clear])
    else:
        mag = operand_magnitude(p, X, tr)
        tol = y_tolerance(X, tr.Y, precision, mag)
        bad = np.abs(Yg - tr.Y) > tol
        assert not bad.any(), f"candidates differ at {np.argwhere(bad)[:5].tolist()}"
        # dormancy / reproduction rows have no transcendental: exact in FP64
        if precision == "fp64":
            dr = (tr.op == 0) | (tr.op == 1)
            assert np.array_equal(Yg[dr], tr.Y[dr])
    # unmoved coordinates are exactly the old ones (masks agree)
    moved_o = tr.Y != np.clip(X, p.lb, p.ub)
    moved_g = Yg != np.clip(X, p.lb, p.ub)
    if precision == "fp64" and p.kind not in ("kapur", "otsu"):
        assert np.array_equal(moved_o, moved_g), "mask / moved coordinates differ"
    prec = "fp32" if bf16 else precision
    ftol = np.array([f_tolerance(p, tr.Y[i], prec) for i in range(p.pop)])
    near = np.abs(tr.Fy - F) <= ftol
    fbad = np.abs(Fyg - tr.Fy) > ftol
    if bf16:
        # a settled row: kept by the GPU, rejected (or a near tie) by the oracle
        settled = fbad & (Fg == F)
        assert np.all(~tr.accepted[settled] | near[settled]), \
            "the BF16 estimate rejected a candidate the oracle accepts"
        fbad &= ~settled
    assert not fbad.any(), \
        f"candidate fitness differs: max {np.max(np.abs(Fyg - tr.Fy) - ftol)}"
    # selection: equal except near ties
    acc_g = ~((Fg == F) & np.all(Xg == X, axis=1)) if bf16 else Fyg < F
    mismatch = (acc_g != tr.accepted) & ~near
    assert not mismatch.any(), f"selection differs at ids {np.where(mismatch)[0][:5]}"
    same = ~near
    mag = operand_magnitude(p, X, tr) if p.kind not in ("kapur", "otsu") else np.zeros_like(X)
    for i in np.where(same)[0]:
        if tr.accepted[i]:
            assert np.all(np.abs(Xg[i] - Xo[i]) <= y_tolerance(X[i], Xo[i], prec, mag[i]))
            assert abs(Fg[i] - Fo[i]) <= ftol[i]
        else:
            assert np.array_equal(Xg[i], X[i]) and Fg[i] == F[i]
    return tr, int(near.sum())

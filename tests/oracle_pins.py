"""Value pins of the oracle's update formulas, as functions of an oracle
library so the same checks can run on the built oracle and on deliberately
altered copies of its source (tests/test_oracle_mutations.py).

Each check returns None when the oracle passes and a short description of
the first disagreement otherwise.  The expected values are the hand-worked
cases of tests/golden/update_formulas.json (the arithmetic is written out
there) and closed forms of Eqs. (4), (7), (9), (10): nothing here calls the
oracle to produce an expected value.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_cases():
    with open(os.path.join(GOLDEN, "update_formulas.json")) as f:
        return json.load(f)["cases"]


def _close(a, b, rel=1e-13):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return a.shape == b.shape and bool(np.all(np.abs(a - b) <= rel * (1.0 + np.abs(b))))


def _problem(case, lib, pdr_plus=False):
    return O.Problem(dim=case["dim"], pop=case["pop"], lb=case["lb"], ub=case["ub"],
                     np_pairs=case["np"], max_iter=case["max_iter"], pf_max=0.0,
                     kind=case.get("kind", "sphere"), pdr_plus=pdr_plus, lib=lib)


def check_case(case, lib=None):
    """One hand-worked case (and its Eq. (13) variant, if it has one)."""
    forms = [(False, case)]
    if "variant_pdr_plus" in case:
        forms.append((True, dict(case, **case["variant_pdr_plus"])))
    for plus, c in forms:
        p = _problem(case, lib, pdr_plus=plus)
        Xn, Fn, tr = p.step_scripted(case["t"], case["X"], case["F"], case["draws"])
        tag = f"{case['name']}{' (variant)' if plus else ''}"
        if tr.op.tolist() != c["expect_op"]:
            return f"{tag}: operations {tr.op.tolist()} != {c['expect_op']}"
        if not _close(tr.Y, c["expect_Y"]):
            return f"{tag}: candidates {tr.Y.tolist()} != {c['expect_Y']}"
        if "expect_Fy" in c and not _close(tr.Fy, c["expect_Fy"]):
            return f"{tag}: candidate fitness {tr.Fy.tolist()}"
        if "expect_accepted" in c and tr.accepted.tolist() != c["expect_accepted"]:
            return f"{tag}: selection {tr.accepted.tolist()} != {c['expect_accepted']}"
        if "expect_X_next" in c and not (_close(Xn, c["expect_X_next"]) and
                                         _close(Fn, c["expect_F_next"])):
            return f"{tag}: next population {Xn.tolist()} {Fn.tolist()}"
    return None


def _forager_draws(pop, dim, r, **own):
    """Every rank an autotroph with an empty mask (its candidate is its
    row), except rank r, which gets `own`."""
    d = [dict(in_dr=False, u_op=0.01, mask=[0] * dim) for _ in range(pop)]
    d[r] = dict(own)
    return d


def check_weight_ratio(lib=None):
    """Eqs. (7) and (10): the pair term is w (X_a - X_b) with w = exp(-|F_a /
    (F_b + eps)|).  With the other terms switched off (X_j = X_i, or Rand = 0
    so that X_near = X_i), two populations with the same rows and order but
    fitness ratios 1/4 and 3/4 move the protozoan by amounts whose ratio is
    exp(-1/4) / exp(-3/4) = exp(1/2) = 1.6487212707001282."""
    want = 1.6487212707001282
    X = np.array([[1.0, 4.0], [0.0, 0.0], [-3.0, 1.0], [2.0, 2.0]])
    moves = {}
    for mode in ("autotroph", "heterotroph"):
        for F in ([1.0, 2.0, 4.0, 5.0], [3.0, 3.5, 4.0, 5.0]):
            p = O.Problem(dim=2, pop=4, lb=-100.0, ub=100.0, np_pairs=1, max_iter=4,
                          pf_max=0.0, lib=lib)
            if mode == "autotroph":
                own = dict(in_dr=False, u_op=0.01, u_f=0.5, j=1, km=[0], kp=[2], mask=[1, 1])
            else:
                own = dict(in_dr=False, u_op=0.99, u_f=0.5, sgn=1, U=[0.0, 0.0], mask=[1, 1])
            _, _, tr = p.step_scripted(1, X, F, _forager_draws(4, 2, 1, **own))
            if tr.op[1] != (2 if mode == "autotroph" else 3):
                return f"{mode}: operation {tr.op[1]}"
            moves.setdefault(mode, []).append(tr.Y[1] - X[1])
        a, b = moves[mode]
        # the move points from X_b to X_a: X_0 - X_2 = (4, 3)
        if not (np.all(a > 0) and np.all(b > 0)):
            return f"{mode}: the pair term does not point from the worse rank to the better"
        if not _close(a / b, [want, want], rel=1e-12):
            return f"{mode}: ratio of moves {(a / b).tolist()} != exp(1/2)"
    return None


def check_foraging_factor(lib=None):
    """Eq. (4): f = rand (1 + cos(pi t / T)).  With the pair weight driven to
    exp(-huge) = 0 (F_k- = -1, F_k+ = 0) and X_j - X_i = (2, -2), an
    autotroph moves by f (2, -2); with rand = 1/2 at t/T = 1/3, 1/2, 2/3 the
    factor is 0.75, 0.5, 0.25 (cos(pi/3) = 1/2, cos(pi/2) = 0,
    cos(2 pi/3) = -1/2)."""
    X = np.array([[5.0, 5.0], [1.0, 3.0], [7.0, -7.0], [3.0, 1.0]])
    F = [-1.0, -0.5, 0.0, 1.0]
    for t, fac in ((2, 0.75), (3, 0.5), (4, 0.25)):
        p = O.Problem(dim=2, pop=4, lb=-100.0, ub=100.0, np_pairs=1, max_iter=6, pf_max=0.0,
                      lib=lib)
        own = dict(in_dr=False, u_op=0.1, u_f=0.5, j=3, km=[0], kp=[2], mask=[1, 1])
        _, _, tr = p.step_scripted(t, X, F, _forager_draws(4, 2, 1, **own))
        if tr.op[1] != 2:
            return f"t={t}: operation {tr.op[1]}"
        if not _close(tr.Y[1], X[1] + fac * np.array([2.0, -2.0])):
            return f"t={t}: candidate {tr.Y[1].tolist()}, factor should be {fac}"
    return None


def check_near_term(lib=None):
    """Eq. (9): X_near = (1 +- Rand (1 - t/T)) X_i.  With the pair weight
    driven to 0, a heterotroph moves by f (X_near - X_i) = f (+-Rand (1 - t/T)
    X_i).  At t/T = 1/2 (f = rand = 1/2), Rand = (1/2, 1/4), X_i = (4, -8):
    sign + gives X_near - X_i = (1, -1) and a move of (0.5, -0.5); sign -
    the opposite.  At t/T = 1/3 (f = 0.75, 1 - t/T = 2/3) with sign + and
    Rand = (3/4, 3/8): X_near - X_i = (2, -2), move (1.5, -1.5)."""
    X = np.array([[9.0, 9.0], [4.0, -8.0], [1.0, 1.0], [2.0, 2.0]])
    F = [-1.0, -0.5, 0.0, 1.0]
    for t, T, U, sgn, move in ((3, 6, [0.5, 0.25], 1, [0.5, -0.5]),
                               (3, 6, [0.5, 0.25], -1, [-0.5, 0.5]),
                               (2, 6, [0.75, 0.375], 1, [1.5, -1.5])):
        p = O.Problem(dim=2, pop=4, lb=-100.0, ub=100.0, np_pairs=1, max_iter=T, pf_max=0.0,
                      lib=lib)
        own = dict(in_dr=False, u_op=0.999, u_f=0.5, sgn=sgn, U=U, mask=[1, 1])
        _, _, tr = p.step_scripted(t, X, F, _forager_draws(4, 2, 1, **own))
        if tr.op[1] != 3:
            return f"t={t}: operation {tr.op[1]}"
        if not _close(tr.Y[1] - X[1], move):
            return f"t={t} sign {sgn}: move {(tr.Y[1] - X[1]).tolist()} != {move}"
    return None


def check_worked_example_finish(lib=None):
    """Section 4.1, Step 6: the printed candidates clamp to the bounds
    (13.53 -> 10), and the strict greedy selection keeps X_1, X_2 and
    replaces X_3, X_4."""
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        g = json.load(f)
    p = O.Problem(dim=g["dim"], pop=g["pop"], lb=g["lb"], ub=g["ub"], pf_max=g["pf_max"],
                  kind="sphere", lib=lib)
    X = np.array(g["step2_sorted_population"])
    F = np.array([p.objective(x) for x in X])
    Xn, _, Yc, _, acc = p.finish(X, F, np.array(g["step5_candidates_by_rank"]))
    if not np.array_equal(Yc, g["step6_clamped_by_rank"]):
        return "clamp differs from the worked example"
    if acc.tolist() != [False, False, True, True]:
        return f"selection {acc.tolist()} differs from the worked example"
    if not np.array_equal(Xn, g["step6_next_population_by_rank"]):
        return "next population differs from the worked example"
    return None


def all_failures(lib=None):
    """Every value pin of the update formulas; the names of those that fail."""
    out = []
    for case in golden_cases():
        msg = check_case(case, lib)
        if msg:
            out.append(msg)
    for chk in (check_weight_ratio, check_foraging_factor, check_near_term,
                check_worked_example_finish):
        msg = chk(lib)
        if msg:
            out.append(f"{chk.__name__}: {msg}")
    return out


__all__ = ["golden_cases", "check_case", "check_weight_ratio", "check_foraging_factor",
           "check_near_term", "check_worked_example_finish", "all_failures", "math"]

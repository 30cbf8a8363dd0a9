"""Value pins of the oracle's update formulas (Section 3): hand-worked
single iterations with every draw fixed through the oracle's scripted-draw
entry point (tests/golden/update_formulas.json, arithmetic written out
there), and closed forms of Eqs. (4), (7), (9), (10).

  Eq. (1) dormancy ............ dormancy_and_reproduction
  Eq. (2) reproduction ........ dormancy_and_reproduction, strict_selection_tie
  Eq. (4) foraging factor ..... every foraging case; check_foraging_factor
  Eq. (6) autotroph ........... autotroph_one_pair, autotroph_two_pairs
  Eq. (7) w_a ................. autotroph_*; check_weight_ratio
  Eq. (8) heterotroph ......... heterotroph_one_pair
  Eq. (9) X_near .............. heterotroph_one_pair; check_near_term
  Eq. (10) w_h ................ heterotroph_one_pair; check_weight_ratio
  Eq. (12) p_ah ............... operation codes of autotroph_one_pair
  Eq. (13) p_dr and its variant dormancy_and_reproduction
  strict selection ............ strict_selection_tie
"""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("case", P.golden_cases(), ids=lambda c: c["name"])
def test_hand_worked_case(case):
    assert P.check_case(case) is None, P.check_case(case)


@pytest.mark.parametrize("check", [P.check_weight_ratio, P.check_foraging_factor,
                                   P.check_near_term, P.check_worked_example_finish],
                         ids=lambda f: f.__name__)
def test_closed_form(check):
    msg = check()
    assert msg is None, msg


def test_scripted_step_equals_drawn_step_when_fed_the_same_draws():
    """The scripted entry runs the same arithmetic as the drawn step: feed it
    the draws the Philox stream produces (read back through the trace and
    the documented mapping) and the candidates agree bit for bit."""
    import numpy as np

    import gen
    import oracle as O
    p = O.Problem(dim=7, pop=9, lb=-5.0, ub=5.0, np_pairs=2, pf_max=1.0, max_iter=10,
                  kind="rastrigin", seed=4)
    X = gen.random_state(9, 7, p.lb, p.ub, 2)
    F = np.array([p.objective(x) for x in X])
    t = 3
    _, _, tr = p.step(t, X, F)
    key = [p.seed & 0xFFFFFFFF, p.seed >> 32]
    draws = []
    for r in range(p.pop):
        idx = int(tr.perm[r])

        def word(tag, q, r=r):
            return int(O.philox4x32_10([(tag << 24) | (q // 4), r, t, 0], key)[q % 4])
        s0 = O.philox4x32_10([(3 << 24) | 0, r, t, 0], key)
        d = dict(in_dr=tr.op[idx] in (0, 1), u_op=O.uniform(s0[0]), u_f=O.uniform(s0[1]),
                 u_rep=O.uniform(s0[2]), sgn=1.0 if O.uniform(s0[3]) < 0.5 else -1.0)
        # the moved coordinates reveal the mask only where the move is nonzero;
        # rebuild it from the keys and the size the trace records
        keys = list(O.philox4x32_10([(3 << 24) | 1, r, t, 0], key)) + \
            list(O.philox4x32_10([(3 << 24) | 2, r, t, 0], key))
        m = int(tr.mcount[idx])
        members = O.subset_mask(p.dim, m, keys)
        d["mask"] = [1 if k in members else 0 for k in range(p.dim)]
        d["U"] = [O.uniform(word(4, k)) for k in range(p.dim)]
        if tr.op[idx] == 2:
            d["j"] = int(tr.nb[idx][0])
            d["km"] = [int(tr.nb[idx][1 + 2 * k]) for k in range(p.np_pairs)]
            d["kp"] = [int(tr.nb[idx][2 + 2 * k]) for k in range(p.np_pairs)]
        draws.append(d)
    _, _, ts = p.step_scripted(t, X, F, draws)
    assert np.array_equal(ts.op, tr.op)
    assert np.array_equal(ts.Y, tr.Y)
    assert np.array_equal(ts.Fy, tr.Fy)

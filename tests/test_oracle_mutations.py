"""The value pins bite: each plausible slip in the update formulas, planted
in a copy of the oracle's source on the CPU (the source itself is never
changed), makes at least one pin of tests/oracle_pins.py fail.

Each mutation replaces one expression of apo_oracle.c that must occur
exactly once; the copy is compiled with the oracle's own flags into a
temporary library and every pin is run against it.
"""
import os
import shutil
import subprocess

import pytest

import oracle as O
import oracle_pins as P
from oracle import build as OB

SRC = os.path.join(os.path.dirname(OB.LIB), "apo_oracle.c")

# (name, expression in the oracle, the slip)
MUTATIONS = [
    ("eq6_pair_sign",
     "wa * (X[(size_t)idm * D + d] - X[(size_t)idp * D + d])",
     "wa * (X[(size_t)idp * D + d] - X[(size_t)idm * D + d])"),
    ("eq7_ratio_swapped",
     "exp(-fabs(F[idm] / (F[idp] + eps)))",
     "exp(-fabs(F[idp] / (F[idm] + eps)))"),
    ("eq7_no_minus",
     "exp(-fabs(F[idm] / (F[idp] + eps)))",
     "exp(fabs(F[idm] / (F[idp] + eps)))"),
    ("eq6_np_dropped",
     "((xj[d] - xi[d]) + acc[d] / (double)np)",
     "((xj[d] - xi[d]) + acc[d])"),
    ("eq6_xj_minus_xi_reversed",
     "((xj[d] - xi[d]) + acc[d] / (double)np)",
     "((xi[d] - xj[d]) + acc[d] / (double)np)"),
    ("eq6_j_ignored",
     "&X[(size_t)perm[dw->j] * D]",
     "&X[(size_t)perm[r] * D]"),
    ("eq8_pair_sign",
     "wh * (X[(size_t)ida * D + d] - X[(size_t)idb * D + d])",
     "wh * (X[(size_t)idb * D + d] - X[(size_t)ida * D + d])"),
    ("eq10_ratio_swapped",
     "exp(-fabs(F[ida] / (F[idb] + eps)))",
     "exp(-fabs(F[idb] / (F[ida] + eps)))"),
    ("eq8_np_dropped",
     "((xnear - xi[d]) + acc[d] / (double)np)",
     "((xnear - xi[d]) + acc[d])"),
    ("eq8_neighbours_not_adjacent",
     "int a = r - k < 0 ? 0 : r - k;",
     "int a = r - 2 * k < 0 ? 0 : r - 2 * k;"),
    ("eq9_additive",
     "(1.0 + (dw->sgn * U[d]) * near_scale) * xi[d]",
     "(1.0 + (dw->sgn * U[d]) * near_scale) + xi[d]"),
    ("eq9_sign_dropped",
     "(1.0 + (dw->sgn * U[d]) * near_scale) * xi[d]",
     "(1.0 + U[d] * near_scale) * xi[d]"),
    ("eq9_t_over_T",
     "const double near_scale = 1.0 - (double)t / (double)T;",
     "const double near_scale = (double)t / (double)T;"),
    ("eq4_minus_cos",
     "const double f_scale = 1.0 + cos(((double)t / (double)T) * OR_PI);",
     "const double f_scale = 1.0 - cos(((double)t / (double)T) * OR_PI);"),
    ("eq4_no_pi",
     "const double f_scale = 1.0 + cos(((double)t / (double)T) * OR_PI);",
     "const double f_scale = 1.0 + cos(((double)t / (double)T));"),
    ("eq4_rand_dropped",
     "const double fac = dw->u_f * f_scale;",
     "const double fac = f_scale;"),
    ("eq2_lower_bound_dropped",
     "double R = p->lb[d] + U[d] * (p->ub[d] - p->lb[d]);",
     "double R = U[d] * (p->ub[d] - p->lb[d]);"),
    ("eq2_rand_dropped",
     "y[d] = xi[d] + (dw->sgn * dw->u_rep) * R;",
     "y[d] = xi[d] + dw->sgn * R;"),
    ("eq2_sign_dropped",
     "y[d] = xi[d] + (dw->sgn * dw->u_rep) * R;",
     "y[d] = xi[d] + dw->u_rep * R;"),
    ("eq1_lower_bound_dropped",
     "y[d] = p->lb[d] + U[d] * (p->ub[d] - p->lb[d]);",
     "y[d] = U[d] * (p->ub[d] - p->lb[d]);"),
    ("eq12_minus_cos",
     "double p_ah = 0.5 * (1.0 + cos(((double)t / (double)T) * OR_PI));",
     "double p_ah = 0.5 * (1.0 - cos(((double)t / (double)T) * OR_PI));"),
    ("eq12_comparison_reversed",
     "return p_ah > dw->u_op ? OR_AUTOTROPH : OR_HETEROTROPH;",
     "return p_ah < dw->u_op ? OR_AUTOTROPH : OR_HETEROTROPH;"),
    ("eq13_sign",
     "p->pdr_plus ? 0.5 * (1.0 + c_dr) : 0.5 * (1.0 - c_dr)",
     "p->pdr_plus ? 0.5 * (1.0 - c_dr) : 0.5 * (1.0 + c_dr)"),
    ("eq13_i_over_ps",
     "double c_dr = cos((1.0 - (double)i / (double)ps) * OR_PI);",
     "double c_dr = cos(((double)i / (double)ps) * OR_PI);"),
    ("mask_ignored_in_foraging",
     "if (mask[d])\n                y[d] = xi[d] + fac",
     "if (1)\n                y[d] = xi[d] + fac"),
    ("selection_not_strict",
     "int acc = Fy[id] < F[id];",
     "int acc = Fy[id] <= F[id];"),
    ("clamp_dropped",
     "y[d] = fmin(fmax(y[d], p->lb[d]), p->ub[d]);",
     "y[d] = y[d];"),
]


def test_pins_pass_on_the_oracle():
    assert P.all_failures() == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_slip_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the expression must occur exactly once"
    mutated = tmp_path / "apo_oracle_mutant.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    subprocess.run([cc, "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-fvisibility=hidden", "-fopenmp", "-o", str(so), str(mutated), "-lm"],
                   check=True, capture_output=True)
    fails = P.all_failures(O.load(str(so)))
    assert fails, f"no pin detects the slip {name}"

"""Plant plausible mistakes in copies of the DGMOC oracle (on the CPU) and check that the
pins of ``test_dgmoc_oracle.py`` catch every one of them."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
C_SRC = os.path.join(ROOT, "oracle", "dgmoc_oracle.c")

MUTANTS = {
    # the axial operator K and the face-driven source
    "K_lower_left_sign": ("-3.0 * f * kap, f * (st + 3.0 * kap)", "3.0 * f * kap, f * (st + 3.0 * kap)"),
    "K_lower_right_factor": ("-3.0 * f * kap, f * (st + 3.0 * kap)", "-3.0 * f * kap, f * (st + kap)"),
    "K_upper_right_dropped": ("double M[4] = {f * (st + kap), f * kap,", "double M[4] = {f * (st + kap), 0.0,"),
    "face_source_dropped": ("double Rv[2] = {f * (q0 + kap * pf), f * (q1 - 3.0 * kap * pf)};",
                            "double Rv[2] = {f * q0, f * q1};"),
    "face_p1_sign": ("f * (q1 - 3.0 * kap * pf)", "f * (q1 + 3.0 * kap * pf)"),
    # segment average
    "average_without_inflow": ("double rhs[2] = {Rv[0] + psi_in[0] - out0, Rv[1] + psi_in[1] - out1};",
                               "double rhs[2] = {Rv[0] - out0, Rv[1] - out1};"),
    # tallies and orientation
    "p1_tally_not_mirrored": ("tal[e + 1] += wdir * l * sgn * bar[1];", "tal[e + 1] += wdir * l * bar[1];"),
    "p1_source_not_mirrored": ("q1 = sgn * src[e + 1] / (4.0 * DGO_PI)", "q1 = src[e + 1] / (4.0 * DGO_PI)"),
    "face_from_average_only": ("next[fi] += o->dlt[a] * l * (bar[0] + bar[1]);", "next[fi] += o->dlt[a] * l * bar[0];"),
    "direction_weight_doubled": ("double kap = o->mu[p] / h, wdir = DGO_PI *", "double kap = o->mu[p] / h, wdir = 2.0 * DGO_PI *"),
    "kappa_uses_sin": ("double kap = o->mu[p] / h,", "double kap = o->sinp[p] / h,"),
    # axial boundary conditions
    "bottom_not_kept": ("if (w == 1) memcpy(o->bot, face, sizeof(double) * nf);", "if (0) memcpy(o->bot, face, sizeof(double) * nf);"),
    "top_always_vacuum": ("} else if (!o->bc_top) {", "} else {"),
    # emission moments
    "p1_scatter_from_p0": ("s += o->sigs[((size_t)m * G + gp) * G + g] * ph[gp * 2 + kk];",
                           "s += o->sigs[((size_t)m * G + gp) * G + g] * ph[gp * 2];"),
    "scatter_transposed": ("s += o->sigs[((size_t)m * G + gp) * G + g] * ph[gp * 2 + kk];",
                           "s += o->sigs[((size_t)m * G + g) * G + gp] * ph[gp * 2 + kk];"),
}


def _probe(so_path):
    """Run every DGMOC oracle pin against an oracle library; True if all hold."""
    code = f"""
import sys
sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {HERE!r})
import oracle.dg_oracle as D
D._SO = {so_path!r}; D._SRC = {so_path!r}
import test_dgmoc_oracle as T
from paper_2607_01591_amd import problems as P
ok = True
# cheapest first; stop at the first pin that fails (a broken oracle may not converge)
cases = [T.test_expm2_matches_scipy]
cases += [lambda c=c: T.test_segment_matches_integrated_ode(c) for c in range(6)]
cases += [T.test_balance_identity_per_sweep]
cases += [lambda b=b: T.test_radially_infinite_slab_equals_1d_dg(*b)
          for b in [(P.BC_VACUUM, P.BC_VACUUM), (P.BC_REFLECTIVE, P.BC_VACUUM), (P.BC_VACUUM, P.BC_REFLECTIVE)]]
cases += [T.test_mirror_symmetric_problem, T.test_tall_planes_reduce_to_planar_moc, T.test_infinite_medium_eigenvalue]
for f in cases:
    try:
        f()
    except (AssertionError, RuntimeError, ValueError, ZeroDivisionError):
        ok = False
        break
print("RESULT", ok)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=900)
    lines = [l for l in r.stdout.splitlines() if l.startswith("RESULT")]
    return bool(lines) and lines[-1].endswith("True")


def _build(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    c.write_text(src_text)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_dgmoc_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(C_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found: {old}"
    so = _build(src.replace(old, new), tmp_path, "mut")
    assert not _probe(so), f"mutant {name} passed every DGMOC pin"


def test_unmutated_dgmoc_oracle_passes(tmp_path):
    so = _build(open(C_SRC).read(), tmp_path, "orig")
    assert _probe(so)

"""Plant plausible mistakes in copies of the DFEM-SN oracle (on the CPU) and check that the
pins of ``test_dfem_oracle.py`` catch every one of them."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
C_SRC = os.path.join(ROOT, "oracle", "dfem_oracle.c")

MUTANTS = {
    "normal_inward": ("o->nx[3 * e + k] = ty / l;", "o->nx[3 * e + k] = -ty / l;"),
    "streaming_sign": ("- (i == 0 ? og[j] * o->area[e] : 0.0)", "+ (i == 0 ? og[j] * o->area[e] : 0.0)"),
    "streaming_transposed": ("- (i == 0 ? og[j] * o->area[e] : 0.0)", "- (j == 0 ? og[i] * o->area[e] : 0.0)"),
    "mass_one_point": ("o->Mm[9 * e + 3 * j + i] += o->area[e] / 3.0 * u[j] * u[i];",
                       "o->Mm[9 * e + 3 * j + i] += (j == 0 && i == 0) ? o->area[e] / 3.0 : 0.0;"),
    "simpson_weights": ("l / 6.0 * (ua[j] * ua[i] + 4.0 * um[j] * um[i] + ub[j] * ub[i])",
                        "l / 3.0 * (ua[j] * ua[i] + um[j] * um[i] + ub[j] * ub[i])"),
    "coupling_own_basis": ("l / 6.0 * (ua[j] * na[i] + 4.0 * um[j] * nm[i] + ub[j] * nb_[i])",
                           "l / 6.0 * (ua[j] * ua[i] + 4.0 * um[j] * um[i] + ub[j] * ub[i])"),
    "mirror_axes_swapped": ("int dm = side < 2 ? o->rx[c->d] : o->ry[c->d];", "int dm = side < 2 ? o->ry[c->d] : o->rx[c->d];"),
    "reflect_not_lagged": ("const double *pm = o->psi_prev + ", "const double *pm = o->psi + "),
    "flux_weight_missing": ("phi[((size_t)e * G + g) * 3 + i] += o->w[d] * ps[i];", "phi[((size_t)e * G + g) * 3 + i] += ps[i];"),
    "slope_scatter_from_average": ("s += o->sigs[((size_t)m * G + gp) * G + g] * phi[((size_t)e * G + gp) * 3 + i];",
                                   "s += o->sigs[((size_t)m * G + gp) * G + g] * phi[((size_t)e * G + gp) * 3];"),
    "source_not_per_steradian": ("q[i] = src[((size_t)e * G + g) * 3 + i] / (4.0 * DFO_PI);", "q[i] = src[((size_t)e * G + g) * 3 + i];"),
}


def _probe(so_path):
    code = f"""
import sys
sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {HERE!r})
import oracle.sn_oracle as S
S._SO = {so_path!r}; S._SRC = {so_path!r}
import test_dfem_oracle as T
ok = True
cases = [lambda d=d: T.test_linear_angular_flux_is_reproduced(d) for d in (0, 3, 5, 10, 13)]
cases += [T.test_mass_matrices_match_numerical_quadrature, T.test_balance_identity_per_sweep, T.test_infinite_medium_eigenvalue, T.test_close_to_planar_moc_on_the_pin_cell]
for f in cases:
    try:
        f()
    except (AssertionError, RuntimeError, ValueError, ZeroDivisionError, FloatingPointError):
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
def test_dfem_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(C_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found: {old}"
    assert not _probe(_build(src.replace(old, new), tmp_path, "mut")), f"mutant {name} passed every DFEM-SN pin"


def test_unmutated_dfem_oracle_passes(tmp_path):
    assert _probe(_build(open(C_SRC).read(), tmp_path, "orig"))

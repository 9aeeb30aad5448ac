"""Plant plausible mistakes in copies of the CMFD oracle (the C current tally and the
Python coarse solve, on the CPU) and check that the pins of ``test_cmfd_oracle.py``
catch every one of them."""
import os
import subprocess
import sys
import types

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
C_SRC = os.path.join(ROOT, "oracle", "moc_oracle.c")
PY_SRC = os.path.join(ROOT, "oracle", "cmfd_oracle.py")

C_MUTANTS = {
    "entry_current_unweighted": ("if (i == 0) jin[(size_t)ci * G + g] += c * psi;", "if (i == 0) jin[(size_t)ci * G + g] += psi;"),
    "crossing_current_unweighted": ("else if (ci != cprev) jpart[coarse_slot(o, cprev, ci) * G + g] += c * psi;",
                                    "else if (ci != cprev) jpart[coarse_slot(o, cprev, ci) * G + g] += psi;"),
    "crossing_reversed": ("else if (ci != cprev) jpart[coarse_slot(o, cprev, ci) * G + g] += c * psi;",
                          "else if (ci != cprev) jpart[coarse_slot(o, ci, cprev) * G + g] += c * psi;"),
    "exit_current_dropped": ("if (o->n_cells && n > 0) jpart", "if (0) jpart"),
}

PY_MUTANTS = {
    "dtilde_sign": ("dt = (-J[s, g] - dh * (phic[j, g] - phic[i, g]))", "dt = (J[s, g] - dh * (phic[j, g] - phic[i, g]))"),
    "dhat_factor": ("dh = L * 2.0 * D[i, g] * D[j, g]", "dh = L * D[i, g] * D[j, g]"),
    "coarse_scatter_transposed": ("-Vc[i] * ssc[i, gp, g]", "-Vc[i] * ssc[i, g, gp]"),
    "coarse_fission_swapped": ("Vc[i] * chic[i, g] * nsfc[i, gp]", "Vc[i] * chic[i, gp] * nsfc[i, g]"),
    "sigma_t_volume_weighted": ("stc = csum(V[:, None] * st * phi) / Vphi", "stc = csum(V[:, None] * st) / Vc[:, None]"),
    "boundary_current_sign": ("dt = J[s, g] / phic[i, g]", "dt = -J[s, g] / phic[i, g]"),
}


def _probe_c(so_path):
    """Run the current-tally pins against an oracle library; True if all hold."""
    code = f"""
import sys
sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {HERE!r})
import oracle.oracle as O
O._SO = {so_path!r}; O._SRC = {so_path!r}
import test_cmfd_oracle as T
ok = True
for name, prob, grid in [(c[0], c[1], c[2]) for c in T.balance_cases()]:
    try:
        T.test_coarse_balance_identity(name, prob, grid)
    except AssertionError:
        ok = False
try:
    T.test_uniform_flux_currents_closed_form()
except AssertionError:
    ok = False
print("RESULT", ok)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    lines = [l for l in r.stdout.splitlines() if l.startswith("RESULT")]
    return bool(lines) and lines[-1].endswith("True")


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_current_tally_mutant_is_caught(name, tmp_path):
    old, new = C_MUTANTS[name]
    src = open(C_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found: {old}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(mut), "-lm"])
    assert not _probe_c(str(so)), f"mutant {name} passed every current pin"


def test_unmutated_current_tally_passes(tmp_path):
    so = tmp_path / "liborc.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), C_SRC, "-lm"])
    assert _probe_c(str(so))


def _py_pins(CM):
    """The coarse-solve pins of test_cmfd_oracle.py, run against module CM."""
    import test_cmfd_oracle as T
    saved = T.CM
    T.CM = CM
    results = {}
    try:
        for name, fn in [("toeplitz", T.test_coarse_operator_toeplitz_eigenvalue),
                         ("kinf", T.test_coarse_operator_infinite_medium_k_inf),
                         ("fixed_point", lambda: T.test_cmfd_reaches_the_power_iteration_fixed_point_faster((1, 0, 1, 0)))]:
            try:
                fn()
                results[name] = True
            except (AssertionError, RuntimeError, np.linalg.LinAlgError, ValueError, ZeroDivisionError):
                results[name] = False
    finally:
        T.CM = saved
    return results


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_coarse_solve_mutant_is_caught(name):
    old, new = PY_MUTANTS[name]
    src = open(PY_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found: {old}"
    mod = types.ModuleType(f"cmfd_mutant_{name}")
    exec(compile(src.replace(old, new), f"<{name}>", "exec"), mod.__dict__)
    res = _py_pins(mod)
    assert not all(res.values()), f"mutant {name} passed every pin: {res}"

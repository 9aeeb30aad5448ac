"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the
pins in ``test_oracle.py`` catch every one of them."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "moc_oracle.c")

MUTANTS = {
    "delta_sign": ("psi -= delta;", "psi += delta;"),
    "expm1_sign": ("(-expm1(-tau))", "(expm1(-tau))"),
    "tau_no_sin": ("o->s_len[k] / o->sinp[p];", "o->s_len[k];"),
    "scatter_transposed": ("o->sigs[((size_t)m * G + gp) * G + g]", "o->sigs[((size_t)m * G + g) * G + gp]"),
    "chi_dropped": ("double v = sc + o->chi[m * G + g] * F / k;", "double v = sc + F / k / G;"),
    "k_not_applied": ("double v = sc + o->chi[m * G + g] * F / k;", "double v = sc + o->chi[m * G + g] * F;"),
    "tally_no_sin": ("o->dlt[a] * o->sinp[p];", "o->dlt[a];"),
    "tally_no_polar_w": ("o->wa[a] * o->wp[p] * o->dlt[a]", "o->wa[a] * o->dlt[a]"),
    "flat_term_no_4pi": ("phi_out[(size_t)r * G + g] = 4.0 * ORC_PI * q[r]",
                         "phi_out[(size_t)r * G + g] = q[r]"),
    "link_wrong_sense": ("size_t j = ((size_t)dst * P + p) * G + g;",
                         "size_t j = ((size_t)(dst ^ 1) * P + p) * G + g;"),
    "k_update": ("knew = k * fs;", "knew = fs;"),
    "merge_without_drop_order": ("if (L < 1e-12) continue;            /* drop first ... */",
                                 "if (L < 1e-3) continue;            /* drop first ... */"),
    "laydown_offset": ("(i + 0.5) * W / o->nx[a]", "(i + 0.25) * W / o->nx[a]"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(mut), "-lm"])
    r = subprocess.run([sys.executable, os.path.join(HERE, "_oracle_probe.py"), str(so)],
                       capture_output=True, text=True, timeout=600)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if not lines:      # the mutant crashed the probe: caught
        return
    res = json.loads(lines[-1])
    assert not all(res.values()), f"mutant {name} passed every pin: {res}"


def test_unmutated_oracle_passes_probe(tmp_path):
    so = tmp_path / "liborc.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), SRC, "-lm"])
    r = subprocess.run([sys.executable, os.path.join(HERE, "_oracle_probe.py"), str(so)],
                       capture_output=True, text=True, timeout=600)
    res = json.loads([l for l in r.stdout.splitlines() if l.startswith("{")][-1])
    assert all(res.values()), res

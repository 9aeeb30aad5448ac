"""Plant plausible mistakes in copies of the HFEM oracle (on the CPU) and check that the
pins of ``test_hfem_oracle.py`` catch every one of them."""
import os
import types

import numpy as np
import pytest

import test_hfem_oracle as T

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "hfem_oracle.py")

MUTANTS = {
    # node integrals
    "stiffness_scale": ("(2.0 / h[e])", "(1.0 / h[e])"),
    "face_coupling_scale": ("* area / 4.0", "* area / 2.0"),
    "face_area_dropped": ("Lam[f * Nfb + m] = area", "Lam[f * Nfb + m] = 1.0"),
    # response matrices (Marshak partial currents)
    "marshak_factor": ("K = np.linalg.inv(2.0 * I + Y)", "K = np.linalg.inv(4.0 * I + Y)"),
    "response_sign": ("K @ (Y - 2.0 * I)", "K @ (2.0 * I - Y)"),
    # cross sections and sources
    "diffusion_coefficient": ("D = 1.0 / (3.0 * self.st[m, g])", "D = 1.0 / self.st[m, g]"),
    "self_scatter_kept": ("sr = self.st[m, g] - self.ss[m, g, g]", "sr = self.st[m, g]"),
    "scatter_transposed": ('np.einsum("nhg,nhi->ngi", ss, phi)', 'np.einsum("ngh,nhi->ngi", ss, phi)'),
    "fission_times_k": ("F[:, None, :] / k", "F[:, None, :] * k"),
    "chi_reversed": ("self.chi[m][:, :, None]", "self.chi[m][:, ::-1, None]"),
    "source_volume_dropped": ("s = self.V[:, None, None] * np.asarray(q, float)", "s = np.asarray(q, float)"),
    # incoming currents and the red-black sweep
    "reflective_as_vacuum": ("jm[~inner, :, sl] = jp[~inner, :, sl]", "pass"),
    "neighbour_same_face": ("jm[inner, :, sl] = jp[self.nbr[inner, f], :, opp]",
                            "jm[inner, :, sl] = jp[self.nbr[inner, f], :, sl]"),
    "red_only": ("for col in (0, 1):", "for col in (0,):"),
    # reconstruction and eigenvalue
    "net_current_sign": ("net = self.jp - self.incoming()", "net = self.incoming() - self.jp"),
    "reconstruct_sign": ('- np.einsum("ngij,ngj->ngi", self.P, net)', '+ np.einsum("ngij,ngj->ngi", self.P, net)'),
    "k_update_inverted": ("self.k = k_old * f_new / f_old", "self.k = k_old * f_old / f_new"),
}


def _pins():
    """Every pin of test_hfem_oracle.py, cheapest first."""
    cases = [T.test_node_integrals_closed_forms]
    cases += [lambda a=a: T.test_quadratic_solution_is_reproduced(a, 2, 1) for a in (2, 0, 1)]
    cases += [T.test_two_group_quadratic_with_up_and_down_scatter, T.test_infinite_medium_eigenvalue,
              T.test_global_balance_with_vacuum_sides, T.test_octant_with_reflective_planes_equals_full_box,
              T.test_bare_box_eigenvalue_converges_to_marshak_diffusion]
    cases += [lambda a=a: T.test_flat_source_slab_converges_to_cosh(a) for a in (2, 0)]
    return cases


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    mod = types.ModuleType("hfem_oracle_mutant")
    exec(compile(src.replace(old, new), f"hfem_oracle[{name}]", "exec"), mod.__dict__)
    monkeypatch.setattr(T, "H", mod)
    caught = False
    with np.errstate(all="ignore"):
        for pin in _pins():
            try:
                pin()
            except Exception:       # an assertion, or a broken oracle failing outright
                caught = True
                break
    assert caught, f"mutant {name} survived every pin"

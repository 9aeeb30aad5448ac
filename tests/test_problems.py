"""Generator invariants: reproducible seeds, valid meshes, cross-section constraints."""
import math

import numpy as np
import pytest

from paper_2607_01591_amd import problems as P


@pytest.mark.parametrize("cfg,target", [(1, 8), (2, 30000), (4, 400000)])
def test_mesh_valid_and_sized(cfg, target):
    p = P.config(cfg)
    a = P.tri_areas(p.xy, p.tri)
    assert (a > 0).all()                                 # counter-clockwise
    assert abs(p.n_regions - target) <= 0.1 * target
    assert np.array_equal(np.unique(p.tri_region), np.arange(p.n_regions))
    assert p.region_material.min() >= 0 and p.region_material.max() < p.n_materials
    # conforming: every interior edge is shared by exactly two triangles
    e = np.sort(np.concatenate([p.tri[:, [0, 1]], p.tri[:, [1, 2]], p.tri[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert cnt.max() == 2
    if p.domain == P.DOMAIN_BOX:
        assert abs(a.sum() - p.box[2] * p.box[3]) < 1e-9 * a.sum()
    else:
        ap = p.hex_apothem
        assert abs(a.sum() - 2 * math.sqrt(3) * ap * ap) < 1e-9 * a.sum()


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_xs_constraints(cfg):
    p = P.config(cfg)
    st, ss, nsf, chi = p.sigma_t, p.sigma_s, p.nu_sigma_f, p.chi
    lo, hi = (0.1, 1.5) if cfg == 4 else (0.2, 2.0)
    assert st.min() >= lo and st.max() <= hi
    ratio = ss.sum(axis=2) / st
    assert ratio.min() >= 0.3 - 1e-12 and ratio.max() <= 0.95 + 1e-12
    sa = st - ss.sum(axis=2)
    assert (sa > 0).all()
    fissile = nsf.sum(axis=1) > 0
    assert fissile.sum() >= 1
    np.testing.assert_allclose(chi[fissile].sum(axis=1), 1.0, rtol=1e-14)
    assert (chi[~fissile] == 0).all()
    r = nsf[fissile] / sa[fissile]
    assert r.min() >= 0.5 and r.max() <= 2.0
    G = p.n_groups
    for m in range(p.n_materials):
        for g in range(G):
            nz = np.nonzero(ss[m, g])[0]
            if cfg == 4:
                assert nz.min() >= g and nz.max() <= g + 6
            else:
                allowed = set(range(g, G)) | ({G - 2} if g == G - 1 else set())
                assert set(nz) <= allowed


def test_seeds_reproducible_and_distinct():
    a, b, c = P.config(2), P.config(2), P.config(2, seed=9)
    assert np.array_equal(a.xy, b.xy) and np.array_equal(a.sigma_t, b.sigma_t)
    assert not np.array_equal(a.sigma_t, c.sigma_t)
    d, e = P.config(5, seed=100001), P.config(5, seed=100002)
    assert np.array_equal(d.xy, e.xy) and np.array_equal(d.tri_region, e.tri_region)
    assert not np.array_equal(d.region_material, e.region_material)


def test_pincell_regions_symmetric():
    p = P.config(1)
    A = p.region_areas()
    np.testing.assert_allclose(A[[0, 2, 4, 4, 4]], A[[1, 3, 5, 6, 7]], rtol=1e-12)
    assert abs(A[:4].sum() - math.pi * 0.54 ** 2) < 1e-12

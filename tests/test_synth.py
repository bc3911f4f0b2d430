"""Checks of the seeded input generators (CPU only)."""
import numpy as np

import hz_synth as syn


def test_centred_sphere_16():
    ph, R2 = syn.centred_sphere(16, 0.2)
    assert R2 == 32.75 and int(ph.sum()) == 840


def test_boolean_spheres_reach_target_and_are_seeded():
    a, ns, vf = syn.boolean_spheres((32, 32, 32), 4.0, 0.3, 9)
    b, ns2, vf2 = syn.boolean_spheres((32, 32, 32), 4.0, 0.3, 9)
    assert np.array_equal(a, b) and ns == ns2
    assert 0.3 <= vf < 0.33 and abs(a.mean() - vf) < 1e-12


def test_rotations_are_proper_orthogonal_and_rotated_cubic_keeps_invariants():
    R = syn.random_rotations(np.random.default_rng(0), 20)
    assert np.abs(np.einsum("nij,nkj->nik", R, R) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-14
    C = syn.cubic_voigt(168.0, 121.0, 75.0)
    s = np.array([1, 1, 1, 2**.5, 2**.5, 2**.5])
    ev = np.sort(np.linalg.eigvalsh(C * np.outer(s, s)))
    for r in R[:5]:
        Cr = syn.rotate_voigt(C, r)
        assert np.abs(np.sort(np.linalg.eigvalsh(Cr * np.outer(s, s))) - ev).max() < 1e-10


def test_voronoi_assigns_every_grain():
    g, _ = syn.voronoi((24, 24, 24), 30, 3)
    assert g.shape == (24, 24, 24) and len(np.unique(g)) == 30

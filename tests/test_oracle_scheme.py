"""Pins of the oracle's Algorithm 1 as a whole (CPU only): the plain-definition
energy minimiser, the laminate closed form, homogeneous special cases, the
real-space force identity of the convergence norm, bounds and symmetries."""
import numpy as np
import pytest

import hz_synth as syn
from oracle import dense, laminate, stencil, tetra, voigt


def _tri_phases(seed, n=3, lo=1.0, hi=5.0):
    rng = np.random.default_rng(seed)
    return np.stack([syn.random_spd_voigt(rng, lo, hi) for _ in range(n)])


def _stiff_ref(C):
    """An isotropic reference with nu = 0 whose modulus exceeds every phase's top eigenvalue."""
    top = max(np.linalg.eigvalsh(c * np.outer([1, 1, 1, 2**.5, 2**.5, 2**.5], [1, 1, 1, 2**.5, 2**.5, 2**.5])).max()
              for c in C)
    return syn.isotropic_voigt(0.75 * top, 0.0)


E_RAND = np.array([1.0, 0.3, -0.2, 0.1, 0.05, -0.3])


def test_dense_minimiser_matches_basic_scheme():
    rng = np.random.default_rng(0)
    ph = rng.integers(0, 3, (6, 4, 4)).astype(np.uint16)
    C = _tri_phases(10)
    d = dense.minimise(ph, C, E_RAND)
    assert d["null_dim"] == 6  # uniform translations of the two FCC corner subgrids
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), E_RAND, tol=1e-14, max_iters=5000)
    assert r.converged
    scale = np.abs(d["mean_sigma"]).max()
    assert np.abs(d["mean_sigma"] - r.mean_sigma).max() < 1e-12 * scale
    # stresses are unique: compare the T1/T2 stress fields pointwise
    assert np.abs(d["sigma_T1"] - r.sigma_T1).max() < 1e-11 * scale
    assert np.abs(d["sigma_T2"] - r.sigma_T2).max() < 1e-11 * scale


def test_dense_minimiser_with_voids_and_eigenstrain():
    rng = np.random.default_rng(1)
    ph = rng.integers(0, 3, (4, 4, 6)).astype(np.uint16)
    C = _tri_phases(11)
    C[2] = 0.0  # voids: zero stiffness is allowed exactly (Sec. 3.2)
    eps0 = np.zeros((3, 6))
    eps0[1] = [0.01, -0.02, 0.005, 0.0, 0.003, 0.0]
    d = dense.minimise(ph, C, E_RAND, eps0=eps0)
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), E_RAND, tol=1e-14, max_iters=20000, eps0=eps0)
    assert r.converged
    scale = np.abs(d["mean_sigma"]).max()
    assert np.abs(d["mean_sigma"] - r.mean_sigma).max() < 1e-11 * scale
    assert np.abs(d["sigma_T1"] - r.sigma_T1).max() < 1e-10 * scale


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_closed_form(axis):
    shape = (6, 8, 10)
    ph = syn.laminate(shape, axis, 3, 7 + axis)
    C = _tri_phases(20 + axis, lo=1.0, hi=30.0)
    fr = [np.mean(ph == k) for k in range(3)]
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), E_RAND, tol=1e-14, max_iters=20000)
    exact = laminate.mean_stress(C, fr, axis, E_RAND)
    assert np.abs(exact - r.mean_sigma).max() < 1e-12 * np.abs(exact).max()


def test_homogeneous_reference_with_eigenstrain_exact_after_one_update():
    """lambda = lambda0 everywhere: the first update of eq. basic_scheme_dep_2 is the
    exact solution, for a fully anisotropic lambda0 (pins Omega = K^-1 index by index)."""
    rng = np.random.default_rng(2)
    C0 = syn.random_spd_voigt(rng, 1.0, 6.0)
    ph = rng.integers(0, 2, (4, 6, 8)).astype(np.uint16)
    eps0 = np.array([[0, 0, 0, 0, 0, 0], [0.02, -0.01, 0.03, 0.004, -0.006, 0.01]])
    C = np.stack([C0, C0])
    r = tetra.basic_scheme(ph, C, C0, E_RAND, fixed_iters=1, eps0=eps0)
    assert r.history[0] > 1e-3
    assert r.history[1] < 1e-14
    d = dense.minimise(ph, C, E_RAND, eps0=eps0)
    assert np.abs(d["mean_sigma"] - r.mean_sigma).max() < 1e-13


def test_homogeneous_without_eigenstrain_is_already_in_equilibrium():
    rng = np.random.default_rng(3)
    C1 = syn.random_spd_voigt(rng, 1.0, 6.0)
    ph = np.zeros((4, 4, 6), dtype=np.uint16)
    r = tetra.basic_scheme(ph, C1[None], _stiff_ref([C1]), E_RAND, tol=1e-12)
    assert r.iters == 0 and r.history[0] < 1e-15
    g = E_RAND * np.array([1, 1, 1, 2, 2, 2])
    assert np.abs(r.mean_sigma - C1 @ g).max() < 1e-14


def test_residual_equals_real_space_force_norm():
    """eq. L2-norm: the q-space norm of r/2 equals the RMS corner force, and
    FT_u(f)(q) = r(q)/2 component by component (Parseval, Sec. 2.6)."""
    rng = np.random.default_rng(4)
    ph = rng.integers(0, 2, (6, 4, 8)).astype(np.uint16)
    C = _tri_phases(30, n=2)
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), E_RAND, fixed_iters=3, keep_spectra=True)
    f = stencil.force(r.sigma_T1, r.sigma_T2)
    L2_real = np.sqrt(np.mean(np.sum(f ** 2, axis=0)))
    assert abs(L2_real - r.L2) < 1e-13 * r.L2
    fq = stencil.corner_FT(f)
    assert np.abs(fq - r.r_hat / 2).max() < 1e-14


def test_algorithm2_equals_algorithm1_every_iteration():
    rng = np.random.default_rng(5)
    ph = rng.integers(0, 2, (6, 6, 4)).astype(np.uint16)
    C = _tri_phases(40, n=2, lo=0.5, hi=8.0)
    C0 = _stiff_ref(C)
    r1 = tetra.basic_scheme(ph, C, C0, E_RAND, fixed_iters=12)
    h2, m2 = tetra.strain_scheme(ph, C, C0, E_RAND, 12)
    assert np.abs(r1.history - h2).max() < 1e-12 * r1.history.max()
    assert np.abs(r1.mean_history - m2).max() < 1e-13


def _ceff(ph, C, C0, tol=1e-12):
    Ce, _ = tetra.effective_stiffness(ph, C, C0, tol=tol, max_iters=20000)
    return Ce


def test_ceff_symmetric_and_between_voigt_and_reuss():
    rng = np.random.default_rng(6)
    ph = rng.integers(0, 2, (6, 6, 6)).astype(np.uint16)
    C = _tri_phases(50, n=2, lo=0.5, hi=10.0)
    Ce = _ceff(ph, C, _stiff_ref(C))
    assert np.abs(Ce - Ce.T).max() < 1e-10 * np.abs(Ce).max()
    f = np.array([np.mean(ph == k) for k in range(2)])
    voigt_b = f[0] * C[0] + f[1] * C[1]
    reuss_b = np.linalg.inv(f[0] * np.linalg.inv(C[0]) + f[1] * np.linalg.inv(C[1]))
    Cs = 0.5 * (Ce + Ce.T)
    assert np.linalg.eigvalsh(voigt_b - Cs).min() > -1e-10
    assert np.linalg.eigvalsh(Cs - reuss_b).min() > -1e-10
    # strictly inside for a genuinely heterogeneous cell
    assert np.linalg.eigvalsh(voigt_b - Cs).max() > 1e-3


def test_ceff_cubic_symmetry_of_centred_sphere():
    ph, _ = syn.centred_sphere(8, 0.2)
    C = np.stack([syn.isotropic_voigt(1.0, 0.3), syn.isotropic_voigt(10.0, 0.3)])
    Ce = _ceff(ph, C, syn.ref_alpha_rule(1.0, 10.0, 0.3))
    s = np.abs(Ce).max()
    for a, b in [((0, 0), (1, 1)), ((0, 0), (2, 2)), ((0, 1), (0, 2)), ((0, 1), (1, 2)),
                 ((3, 3), (4, 4)), ((3, 3), (5, 5))]:
        assert abs(Ce[a] - Ce[b]) < 1e-10 * s
    off = Ce.copy()
    off[:3, :3] = 0
    off[[3, 4, 5], [3, 4, 5]] = 0
    assert np.abs(off).max() < 1e-10 * s


def test_ceff_invariant_under_translation_and_reflection():
    rng = np.random.default_rng(7)
    ph = rng.integers(0, 2, (4, 6, 8)).astype(np.uint16)
    C = np.stack([syn.isotropic_voigt(1.0, 0.25), syn.isotropic_voigt(7.0, 0.25)])
    C0 = syn.ref_alpha_rule(1.0, 7.0, 0.25)
    Ce = _ceff(ph, C, C0)
    Ct = _ceff(np.roll(ph, (1, -2, 3), axis=(0, 1, 2)), C, C0)
    assert np.abs(Ce - Ct).max() < 1e-10 * np.abs(Ce).max()
    # mirror x1 -> -x1: components with an odd number of index 1 change sign
    Cr = _ceff(ph[:, :, ::-1].copy(), C, C0)
    sign = np.array([1, 1, 1, 1, -1, -1])  # Voigt 11,22,33,23,13,12: parity of index 1
    assert np.abs(Cr - np.outer(sign, sign) * Ce).max() < 1e-10 * np.abs(Ce).max()


def test_sphere16_converges_well_under_hundred_iterations():
    """The 16^3 sphere (20% vf, contrast 10) converges to 1e-8 with the alpha-rule
    reference; soft check only: the paper prints iteration counts only in figures."""
    p = syn.sphere16()
    r = tetra.basic_scheme(p.phase, p.C, p.C0, p.loads[0], tol=p.tol, keep_fields=False)
    assert r.converged and r.iters < 100
    assert r.max_imag < 1e-15

"""Pins of the oracle's applied-stress loop (Sec. 2.5, step 6 of Algorithm 1) and
of eigenstrains, CPU only: the energy minimiser with the external-work term, closed
forms for homogeneous cells, and the identity that turns step 6 into a correction
by the mean-stress mismatch."""
import numpy as np

import hz_synth as syn
from oracle import dense, tetra, voigt

S_A = np.array([0.5, -0.2, 0.1, 0.05, 0.0, 0.3])
EPS0 = np.array([[0, 0, 0, 0, 0, 0], [0.01, -0.02, 0.005, 0.0, 0.003, 0.0], [0, 0, 0, 0, 0, 0]])
MANDEL = np.array([1, 1, 1, 2**.5, 2**.5, 2**.5])


def _phases(seed, n=3, lo=1.0, hi=5.0):
    rng = np.random.default_rng(seed)
    return np.stack([syn.random_spd_voigt(rng, lo, hi) for _ in range(n)])


def _stiff_ref(C):
    top = max(np.linalg.eigvalsh(c * np.outer(MANDEL, MANDEL)).max() for c in C)
    return syn.isotropic_voigt(0.75 * top, 0.0)


def _mandel(Cv):
    return np.asarray(Cv) * np.outer(MANDEL, MANDEL)


def test_solve_stiffness_inverts_the_double_contraction():
    rng = np.random.default_rng(0)
    Cv = syn.random_spd_voigt(rng, 0.5, 4.0)
    X = voigt.sym_tensor(rng.normal(size=6))
    Y = np.einsum("ijkl,kl->ij", voigt.stiffness_tensor(Cv), X)
    assert np.abs(voigt.solve_stiffness(Cv, Y) - X).max() < 1e-14 * np.abs(X).max()


def test_stress_loading_matches_energy_minimiser_with_eigenstrain():
    """The converged stress-loaded iterate minimises the functional with the
    external work: <sigma> = sigma^a, the same Ebar and the same stress fields."""
    rng = np.random.default_rng(1)
    ph = rng.integers(0, 3, (4, 4, 6)).astype(np.uint16)
    C = _phases(1)
    d = dense.minimise(ph, C, S_A, eps0=EPS0, stress=True)
    assert np.abs(d["mean_sigma"] - S_A).max() < 1e-13
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), S_A, tol=1e-13, max_iters=20000, eps0=EPS0, stress=True)
    assert r.converged
    scale = np.abs(S_A).max()
    assert np.abs(r.mean_sigma - S_A).max() < 1e-12 * scale
    assert np.abs(r.Ebar - d["Ebar"]).max() < 1e-12 * np.abs(d["Ebar"]).max()
    assert np.abs(r.sigma_T1 - d["sigma_T1"]).max() < 1e-12 * scale
    assert np.abs(r.sigma_T2 - d["sigma_T2"]).max() < 1e-12 * scale


def test_stress_loading_with_voids():
    rng = np.random.default_rng(2)
    ph = rng.integers(0, 3, (6, 4, 4)).astype(np.uint16)
    ph[0] = 0  # a stiff layer keeps the cell load-bearing in every direction
    C = _phases(2)
    C[2] = 0.0
    d = dense.minimise(ph, C, S_A, stress=True)
    r = tetra.basic_scheme(ph, C, _stiff_ref(C), S_A, tol=1e-12, max_iters=50000, stress=True)
    assert r.converged
    assert np.abs(r.Ebar - d["Ebar"]).max() < 1e-9 * np.abs(d["Ebar"]).max()
    assert np.abs(r.mean_sigma - S_A).max() < 1e-11


def test_strain_solve_at_the_converged_mean_strain_reproduces_the_stress_solve():
    rng = np.random.default_rng(3)
    ph = rng.integers(0, 3, (6, 6, 4)).astype(np.uint16)
    C = _phases(3)
    C0 = _stiff_ref(C)
    rs = tetra.basic_scheme(ph, C, C0, S_A, tol=1e-13, max_iters=20000, eps0=EPS0, stress=True)
    re = tetra.basic_scheme(ph, C, C0, rs.Ebar, tol=1e-13, max_iters=20000, eps0=EPS0)
    assert np.abs(re.mean_sigma - S_A).max() < 1e-12
    assert np.abs(re.sigma_T1 - rs.sigma_T1).max() < 1e-12


def test_step6_equals_mean_stress_correction():
    """With <lambda:deps> + <lambda>:Ebar - <lambda:eps0> = <sigma>, step 6 reads
    Ebar_{k+1} = Ebar_k + lambda0^-1:(sigma^a - <sigma>_k); checked on every step of a
    heterogeneous anisotropic cell with eigenstrain and an anisotropic reference."""
    rng = np.random.default_rng(4)
    ph = rng.integers(0, 3, (4, 6, 8)).astype(np.uint16)
    C = _phases(4)
    C0 = syn.random_spd_voigt(rng, 5.0, 9.0)
    r = tetra.basic_scheme(ph, C, C0, S_A, fixed_iters=8, eps0=EPS0, stress=True)
    S0 = np.linalg.inv(_mandel(C0))
    for k in range(8):
        step = (r.Ebar_history[k + 1] - r.Ebar_history[k]) * MANDEL
        want = S0 @ ((S_A - r.mean_history[k]) * MANDEL)
        assert np.abs(step - want).max() < 1e-14 * np.abs(want).max() + 1e-17
    assert np.abs(r.Ebar_history[0] * MANDEL - S0 @ (S_A * MANDEL)).max() < 1e-15


def test_homogeneous_cell_mean_strain_follows_the_linear_recursion():
    """lambda uniform: u stays zero, and Ebar_n - Ebar* = (I - S0 lambda)^n (Ebar_0 - Ebar*)
    with Ebar* = lambda^-1:sigma^a (Mandel basis)."""
    rng = np.random.default_rng(5)
    Cv = syn.random_spd_voigt(rng, 1.0, 4.0)
    C0 = _stiff_ref([Cv])
    ph = np.zeros((4, 6, 4), dtype=np.uint16)
    n = 12
    r = tetra.basic_scheme(ph, Cv[None], C0, S_A, fixed_iters=n, stress=True)
    assert np.abs(r.u_hat).max() == 0.0
    M, M0 = _mandel(Cv), _mandel(C0)
    e_star = np.linalg.solve(M, S_A * MANDEL)
    G = np.eye(6) - np.linalg.solve(M0, M)
    e0 = np.linalg.solve(M0, S_A * MANDEL)
    for k in range(n + 1):
        want = e_star + np.linalg.matrix_power(G, k) @ (e0 - e_star)
        assert np.abs(r.Ebar_history[k] * MANDEL - want).max() < 1e-14 * np.abs(e_star).max()


def test_eigenstrain_inclusion_under_zero_stress_homogeneous_elasticity():
    """sigma^a = 0, lambda uniform, eigenstrain in part of the cell: the mean strain is
    the mean eigenstrain exactly (<sigma> = lambda:(Ebar - <eps0>) = 0), and the fields
    equal the strain-loaded solution at that mean strain (Sec. 3.3 set-up)."""
    Cv = syn.isotropic_voigt(2.0, 0.3)
    ph = np.zeros((8, 8, 8), dtype=np.uint16)
    ph[2:5, 3:6, 1:4] = 1
    C = np.stack([Cv, Cv])
    e0 = np.array([[0, 0, 0, 0, 0, 0], [0.0, 0.0, 0.01, 0.0, 0.0, 0.0]])
    C0 = syn.isotropic_voigt(2.6, 0.0)
    r = tetra.basic_scheme(ph, C, C0, np.zeros(6), tol=1e-12, max_iters=5000, eps0=e0, stress=True)
    assert r.converged
    f = np.mean(ph == 1)
    assert np.abs(r.Ebar - f * e0[1]).max() < 1e-14
    assert np.abs(r.mean_sigma).max() < 1e-13
    re = tetra.basic_scheme(ph, C, C0, f * e0[1], tol=1e-12, max_iters=5000, eps0=e0)
    assert np.abs(re.sigma_T1 - r.sigma_T1).max() < 1e-12
    # the stop-rule scale is the eigenstress norm when sigma^a = 0
    Ce0 = voigt.frobenius(f * np.einsum("ijkl,kl->ij", voigt.stiffness_tensor(Cv), voigt.sym_tensor(e0[1])))
    assert abs(r.history[-1] * Ce0 - r.L2) < 1e-12 * r.L2 + 1e-300


def test_cubic_void_under_pressure_converges_as_the_paper_reports():
    """Sec. 3.2 workload (31^3 void in 64^3, mu = 132.30 GPa, nu = 0.26, P = 300 MPa,
    lambda0 = 0.8 lambda_m): the paper reaches eps = 1e-10 in fewer than 100 iterates
    (read from its convergence figure; a soft pin of the whole applied-stress path)."""
    N = 64
    ph = np.zeros((N, N, N), dtype=np.uint16)
    ph[16:47, 16:47, 16:47] = 1
    mu, nu = 132.30e3, 0.26
    Cm = syn.isotropic_voigt(2.0 * mu * (1.0 + nu), nu)
    C = np.stack([Cm, np.zeros((6, 6))])
    sa = np.array([-300.0, -300.0, -300.0, 0.0, 0.0, 0.0])
    r = tetra.basic_scheme(ph, C, 0.8 * Cm, sa, tol=1e-10, max_iters=200, stress=True, keep_fields=False)
    assert r.converged and r.iters < 100
    assert np.abs(r.mean_sigma - sa).max() < 1e-10 * 300 * np.sqrt(3)

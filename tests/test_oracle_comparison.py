"""Pins of the oracle's comparison Green operators (CPU only): the rotated symbol
against the tetrahedral one and against its real-space differences, the zero
sets, the continuous symbol against the textbook periodic spectral
differentiation matrix, the strain Green operator against the isotropic closed
form, exactness after one update, and the laminate closed form."""
import numpy as np
import pytest

import hz_synth as syn
from oracle import comparison as cmp_
from oracle import laminate, tetra, voigt

SHAPE = (6, 8, 10)
E_RAND = np.array([1.0, 0.3, -0.2, 0.1, 0.05, -0.3])


def test_rotated_symbol_is_the_average_of_the_tetrahedral_gradients():
    """The 8-corner rotated gradient is the mean of the two tetrahedral gradients
    D^T1 = D, D^T2 = -conj(D) (Sec. 2.2), up to the phase exp(i(q1+q2+q3)/2) that the
    footnote of Appendix B attaches to a displacement grid shifted by half a voxel."""
    q1, q2, q3 = tetra.qvectors(SHAPE)
    D = tetra.D_symbol(SHAPE)
    Dr = cmp_.rotated_symbol(SHAPE)
    ph = np.exp(-0.5j * (q1 + q2 + q3))
    assert np.abs(Dr * ph - 0.5 * (D - np.conj(D))).max() < 1e-15


def test_rotated_symbol_is_its_real_space_difference():
    """(D_1 f)(r) = 1/4 sum over the 4 cube edges along x of f(r + e1 + b) - f(r + b),
    b in {0, e2, e3, e2 + e3}; likewise along y and z (eq. Dq_rotated in real space)."""
    rng = np.random.default_rng(0)
    f = rng.standard_normal(SHAPE[::-1])
    spec = tetra.FT(f)
    Dr = cmp_.rotated_symbol(SHAPE)
    ax = {0: -1, 1: -2, 2: -3}  # tensor axis -> array axis
    for i in range(3):
        got = tetra.FTinv(Dr[i] * spec).real
        want = np.zeros_like(f)
        others = [j for j in range(3) if j != i]
        for b in range(2):
            for c in range(2):
                g = np.roll(f, -b, axis=ax[others[0]])
                g = np.roll(g, -c, axis=ax[others[1]])
                want += 0.25 * (np.roll(g, -1, axis=ax[i]) - g)
        assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("shape", [(6, 8, 10), (4, 6, 8), (8, 4, 6)])
def test_zero_sets_are_the_masks(shape):
    for name, (sym, mask) in cmp_.OPERATORS.items():
        D = sym(shape)
        zero = np.sum(np.abs(D) ** 2, axis=0) < 1e-28
        assert np.array_equal(zero, mask(shape)), name
    # the rotated scheme vanishes on three lines through (pi,pi,pi) (Appendix B)
    N1, N2, N3 = shape
    assert cmp_.rotated_singular(shape).sum() == 1 + N1 + N2 + N3 - 2


@pytest.mark.parametrize("N", [8, 10, 12])
def test_continuous_symbol_is_the_periodic_spectral_derivative(N):
    """On an even grid of unit spacing the derivative of the band-limited interpolant
    at the nodes is the circulant with entries (pi/N)(-1)^m cot(pi m / N), m != 0
    (Trefethen, Spectral Methods in MATLAB, ch. 3); its highest mode is a cosine
    whose derivative vanishes at the nodes, which is the reading xi(N/2) = 0."""
    shape = (N, 4, 6)
    rng = np.random.default_rng(N)
    f = rng.standard_normal(shape[::-1])
    D = cmp_.continuous_symbol(shape)
    got = tetra.FTinv(D[0] * tetra.FT(f)).real
    m = np.arange(N)
    col = np.zeros(N)
    col[1:] = (np.pi / N) * (-1.0) ** m[1:] / np.tan(np.pi * m[1:] / N)
    # (Df)(x) = sum_m c(m) f(x - m)... with c(m) = -col(m): d/dx at node x of the interpolant
    M = np.array([[(-col[(k - j) % N]) if k != j else 0.0 for k in range(N)] for j in range(N)])
    want = np.einsum("jk,abk->abj", M, f)
    assert np.abs(got - want).max() < 1e-12
    # a band-limited sine is differentiated exactly
    x = np.arange(N)
    g = np.broadcast_to(np.sin(2 * np.pi * 3 * x / N), shape[::-1])
    dg = tetra.FTinv(D[0] * tetra.FT(g)).real
    assert np.abs(dg - 2 * np.pi * 3 / N * np.cos(2 * np.pi * 3 * x / N)).max() < 1e-12
    # the alternating mode is not a gradient
    alt = np.broadcast_to((-1.0) ** x, shape[::-1])
    assert np.abs(tetra.FTinv(D[0] * tetra.FT(alt))).max() < 1e-12


@pytest.mark.parametrize("operator", ["rotated", "continuous"])
def test_strain_green_operator_matches_the_isotropic_closed_form(operator):
    """For D = i k exp(i phi) with k real, D (x)_s Omega (sigma.conj D) is the classical
    isotropic strain Green operator of the frequency vector k:
    Gamma_khij = [d_ki k_h k_j + d_hi k_k k_j + d_kj k_h k_i + d_hj k_k k_i]/(4 mu0 |k|^2)
               - (lam0 + mu0)/(mu0 (lam0 + 2 mu0)) k_i k_j k_k k_h / |k|^4."""
    shape = (6, 8, 4)
    sym, mask = cmp_.OPERATORS[operator]
    D = sym(shape)
    lam0, mu0 = 1.7, 0.9
    C0 = np.zeros((6, 6))
    C0[:3, :3] = lam0
    C0[np.arange(3), np.arange(3)] += 2 * mu0
    C0[np.arange(3, 6), np.arange(3, 6)] = mu0
    Om = cmp_.green(D, voigt.stiffness_tensor(C0), mask(shape))
    rng = np.random.default_rng(1)
    s = rng.standard_normal((3, 3) + shape[::-1]) + 1j * rng.standard_normal((3, 3) + shape[::-1])
    s = 0.5 * (s + np.swapaxes(s, 0, 1))
    got = tetra.sym_outer(D, np.einsum("il...,l...->i...", Om, tetra.dot_vec(s, np.conj(D))))
    # k: D = i k e^{i phi}, so k = Im(D e^{-i phi}) with the phase of the largest component
    m = mask(shape)
    big = np.argmax(np.abs(D), axis=0)
    Dbig = np.take_along_axis(D, big[None], axis=0)[0]
    phase = np.where(m, 1.0, Dbig / np.where(m, 1.0, 1j * np.abs(Dbig)))
    k = np.real(D / (1j * phase))
    assert np.abs(np.imag(D / (1j * phase))).max() < 1e-13
    k2 = np.where(m, 1.0, np.sum(k * k, axis=0))
    d = np.eye(3)
    t1 = (np.einsum("ki,h...,j...->khij...", d, k, k) + np.einsum("hi,k...,j...->khij...", d, k, k)
          + np.einsum("kj,h...,i...->khij...", d, k, k) + np.einsum("hj,k...,i...->khij...", d, k, k))
    G = t1 / (4 * mu0 * k2) - (lam0 + mu0) / (mu0 * (lam0 + 2 * mu0)) * np.einsum(
        "i...,j...,k...,h...->khij...", k, k, k, k) / k2 ** 2
    want = np.einsum("khij...,ij...->kh...", G, s)
    want[:, :, m] = 0.0
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("operator", ["rotated", "continuous"])
def test_homogeneous_reference_with_eigenstrain_exact_after_one_update(operator):
    """lambda = lambda0 everywhere (fully anisotropic): the first update solves the
    problem, so the residual of iterate 1 vanishes (pins Omega = K^-1 index by index,
    and Omega := 0 where D vanishes costs nothing there)."""
    rng = np.random.default_rng(2)
    C0 = syn.random_spd_voigt(rng, 1.0, 6.0)
    ph = rng.integers(0, 2, (4, 6, 8)).astype(np.uint16)
    eps0 = np.array([[0, 0, 0, 0, 0, 0], [0.02, -0.01, 0.03, 0.004, -0.006, 0.01]])
    r = cmp_.basic_scheme(ph, np.stack([C0, C0]), C0, E_RAND, operator, fixed_iters=1, eps0=eps0)
    assert r.history[0] > 1e-3
    assert r.history[1] < 1e-14
    assert r.max_imag < 1e-13


def _even_layers(shape, axis, seed):
    """Three phases in layers of even thickness starting at even planes."""
    rng = np.random.default_rng(seed)
    n = shape[axis]
    lab = np.repeat(rng.integers(0, 3, n // 2), 2)
    lab[:2], lab[2:4] = 0, 1  # every phase present
    lab[4:6] = 2
    full = np.empty(shape[::-1], dtype=np.uint16)
    sl = [np.newaxis] * 3
    sl[2 - axis] = slice(None)
    full[...] = lab[tuple(sl)]
    return full


@pytest.mark.parametrize("operator", ["rotated", "continuous"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_closed_form(operator, axis):
    """With the stiffness a function of x_n, both gradients reduce to a one-dimensional
    difference (rotated) or derivative (continuous) along n, and with layers of even
    thickness the laminate's piecewise-uniform strain has no component at the highest
    frequency: both schemes reach the continuum laminate exactly."""
    shape = (8, 10, 12)
    ph = _even_layers(shape, axis, 7 + axis)
    rng = np.random.default_rng(20 + axis)
    C = np.stack([syn.random_spd_voigt(rng, 1.0, 30.0) for _ in range(3)])
    top = max(np.linalg.eigvalsh(c * np.outer([1, 1, 1, 2**.5, 2**.5, 2**.5],
                                              [1, 1, 1, 2**.5, 2**.5, 2**.5])).max() for c in C)
    C0 = syn.isotropic_voigt(0.75 * top, 0.0)
    r = cmp_.basic_scheme(ph, C, C0, E_RAND, operator, tol=1e-13, max_iters=20000)
    assert r.converged
    fr = [np.mean(ph == k) for k in range(3)]
    exact = laminate.mean_stress(C, fr, axis, E_RAND)
    assert np.abs(exact - r.mean_sigma).max() < 1e-11 * np.abs(exact).max()


def test_rotated_and_tetrahedral_schemes_differ_off_laminates():
    """The three discretisations are different problems: on a random two-phase cell
    their converged <sigma> differ by far more than the tolerance, yet each lies
    between the soft phase's Young modulus and the Voigt average of C11."""
    rng = np.random.default_rng(3)
    ph = rng.integers(0, 2, (6, 6, 6)).astype(np.uint16)
    C = np.stack([syn.isotropic_voigt(1.0, 0.3), syn.isotropic_voigt(10.0, 0.3)])
    C0 = syn.isotropic_voigt(5.95, 0.3)
    E = np.array([1.0, 0, 0, 0, 0, 0])
    t = tetra.basic_scheme(ph, C, C0, E, tol=1e-12, max_iters=5000, keep_fields=False)
    res = {"tetra": t.mean_sigma[0]}
    for op in ("rotated", "continuous"):
        r = cmp_.basic_scheme(ph, C, C0, E, op, tol=1e-12, max_iters=5000)
        assert r.converged
        res[op] = r.mean_sigma[0]
    f = np.mean(ph == 1)
    voigt_11 = (1 - f) * C[0][0, 0] + f * C[1][0, 0]
    for v in res.values():
        assert 1.0 < v < voigt_11
    assert abs(res["rotated"] - res["tetra"]) > 1e-6
    assert abs(res["continuous"] - res["tetra"]) > 1e-6

"""Pins of the oracle's transforms, Fourier symbols and Green operators (CPU only).

Each test compares the oracle with something other than itself: naive DFT
sums, closed forms derived by hand, the real-space stencils of eqs. DA1-DA2,
and invariants the paper states."""
import numpy as np
import pytest

import hz_synth as syn
from oracle import stencil, tetra, voigt


def naive_FT(a):
    """(1/N) sum_r a(r) exp(-i q.r), written as a direct sum (eq. FT)."""
    N3, N2, N1 = a.shape
    l3, l2, l1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    out = np.zeros(a.shape, dtype=complex)
    for h3 in range(N3):
        for h2 in range(N2):
            for h1 in range(N1):
                ph = 2 * np.pi * (h1 * l1 / N1 + h2 * l2 / N2 + h3 * l3 / N3)
                out[h3, h2, h1] = np.sum(a * np.exp(-1j * ph)) / a.size
    return out


def test_ft_matches_naive_sum_mixed_radix():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((10, 6, 4)) + 1j * rng.standard_normal((10, 6, 4))
    A = tetra.FT(a)
    assert np.max(np.abs(A - naive_FT(a))) < 1e-14
    # inverse transform is unnormalised: sum_q A(q) exp(+i q.r)
    back = tetra.FTinv(A)
    assert np.max(np.abs(back - a)) < 1e-13
    assert abs(A[0, 0, 0] - a.mean()) < 1e-15


@pytest.mark.parametrize("shape", [(8, 6, 10), (4, 4, 6), (16, 12, 2)])
def test_D_norm_closed_form_and_zero_set(shape):
    D = tetra.D_symbol(shape)
    q1, q2, q3 = tetra.qvectors(shape)
    # |D|^2 = 4 [1 - prod cos^2(q_j/2) - prod sin^2(q_j/2)]
    closed = 4 * (1 - (np.cos(q1 / 2) * np.cos(q2 / 2) * np.cos(q3 / 2)) ** 2
                  - (np.sin(q1 / 2) * np.sin(q2 / 2) * np.sin(q3 / 2)) ** 2)
    n2 = np.sum(np.abs(D) ** 2, axis=0)
    assert np.max(np.abs(n2 - closed)) < 1e-14
    # D vanishes exactly at h = 0 and h = N/2 (Sec. 2.2), nowhere else
    zeros = np.argwhere(n2 < 1e-20)
    N1, N2, N3 = shape
    assert sorted(map(tuple, zeros)) == sorted([(0, 0, 0), (N3 // 2, N2 // 2, N1 // 2)])
    assert np.all(tetra.singular_mask(shape) == (n2 < 1e-20))


@pytest.mark.parametrize("tet", [1, 2])
def test_symbol_equals_real_space_stencil(tet):
    """D (x)_s u in q-space equals the 4-corner stencil of eqs. DA1-DA2 in real space."""
    shape = (6, 8, 4)
    N1, N2, N3 = shape
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, N3, N2, N1))  # corner displacements, integer-indexed corners
    uq = stencil.corner_FT(u)  # paper's transform over corner positions (eq. FT_u)
    D = tetra.D_symbol(shape)
    sym = D if tet == 1 else -np.conj(D)  # eqs. desp_T1_dep_Q, desp_T2_dep_Q
    eq = tetra.sym_outer(sym, uq)
    er = tetra.FTinv(eq)
    assert np.max(np.abs(er.imag)) < 1e-13
    assert np.max(np.abs(er.real - stencil.grad(u, tet))) < 1e-13


def iso_K(D, lam, mu):
    """K = 2 mu |D|^2 I + 2 (lam + mu)(a a^T + b b^T), D = a + i b (derived by hand)."""
    a, b = D.real, D.imag
    n2 = np.sum(np.abs(D) ** 2, axis=0)
    K = 2 * (lam + mu) * (np.einsum("i...,j...->ij...", a, a) + np.einsum("i...,j...->ij...", b, b))
    for i in range(3):
        K[i, i] += 2 * mu * n2
    return K


def test_green_isotropic_closed_form():
    shape = (8, 6, 10)
    E, nu = 3.0, 0.27
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C0t = voigt.stiffness_tensor(syn.isotropic_voigt(E, nu))
    D = tetra.D_symbol(shape)
    K = tetra.green_inverse(D, C0t)
    assert np.max(np.abs(K - iso_K(D, lam, mu))) < 1e-13
    Om = tetra.green(D, C0t, shape)
    prod = np.einsum("ij...,jk...->ik...", Om, iso_K(D, lam, mu))
    mask = tetra.singular_mask(shape)
    eye = np.eye(3)[:, :, None, None, None]
    assert np.max(np.abs((prod - eye)[:, :, ~mask])) < 1e-12
    assert np.all(Om[:, :, mask] == 0)


def test_green_real_symmetric_and_pi_periodic():
    """Omega real symmetric (eq. displacement_Green_function_symmetry) and
    Omega(q + (pi,pi,pi)) = Omega(q) (eq. Fourier_component_relations_4)."""
    shape = (8, 6, 10)
    rng = np.random.default_rng(3)
    C0 = syn.random_spd_voigt(rng, 1.0, 4.0)
    C0t = voigt.stiffness_tensor(C0)
    Om = tetra.green(tetra.D_symbol(shape), C0t, shape)
    assert np.max(np.abs(Om - np.swapaxes(Om, 0, 1))) < 1e-14 * np.max(np.abs(Om))
    shifted = np.roll(Om, shift=(-5, -3, -4), axis=(-3, -2, -1))
    assert np.max(np.abs(shifted - Om)) < 1e-12 * np.max(np.abs(Om))


def _pair_green(q, C0t):
    D = tetra.D_at(*q)
    K = tetra.green_inverse(D, C0t).real
    Om = np.moveaxis(np.linalg.inv(np.moveaxis(K, (0, 1), (-2, -1))), (-2, -1), (0, 1))
    return D, Om, tetra.strain_green(D, Om)


def test_pair_green_idempotent_off_lattice():
    """G Lambda0 G = G for the T1/T2 pair operator G = [[G^d, G^nd], [conj G^nd, conj G^d]]."""
    rng = np.random.default_rng(4)
    C0t = voigt.stiffness_tensor(syn.random_spd_voigt(rng, 1.0, 5.0))
    q = [rng.uniform(0.01, 2 * np.pi - 0.01, 64) for _ in range(3)]
    D, Om, (Gd, Gnd, _) = _pair_green(q, C0t)
    G = [[Gd, Gnd], [np.conj(Gnd), np.conj(Gd)]]

    def c(A, B):
        return np.einsum("ijkl...,klmn...,mnpr...->ijpr...", A, C0t[..., None], B)

    for a in range(2):
        for b in range(2):
            GLG = c(G[a][0], G[0][b]) + c(G[a][1], G[1][b])
            assert np.max(np.abs(GLG - G[a][b])) < 1e-12 * np.max(np.abs(G[a][b]))


def test_strain_green_identities_and_symmetries():
    """G^d:l0:de1 + G^nd:l0:de2 = de1 and the conjugate relation (Sec. 2.6), and the
    index symmetries of G^d, G^nd."""
    rng = np.random.default_rng(5)
    C0t = voigt.stiffness_tensor(syn.random_spd_voigt(rng, 1.0, 5.0))
    q = [rng.uniform(0.01, 2 * np.pi - 0.01, 32) for _ in range(3)]
    D, Om, (Gd, Gnd, Gam) = _pair_green(q, C0t)
    u = rng.standard_normal((3, 32)) + 1j * rng.standard_normal((3, 32))
    de1 = tetra.sym_outer(D, u)
    de2 = tetra.sym_outer(-np.conj(D), u)
    s1 = np.einsum("ijkl,kl...->ij...", C0t, de1)
    s2 = np.einsum("ijkl,kl...->ij...", C0t, de2)
    lhs1 = np.einsum("ijkl...,kl...->ij...", Gd, s1) + np.einsum("ijkl...,kl...->ij...", Gnd, s2)
    lhs2 = (np.einsum("ijkl...,kl...->ij...", np.conj(Gnd), s1)
            + np.einsum("ijkl...,kl...->ij...", np.conj(Gd), s2))
    assert np.max(np.abs(lhs1 - de1)) < 1e-12
    assert np.max(np.abs(lhs2 - de2)) < 1e-12
    assert np.allclose(Gd, np.swapaxes(Gd, 0, 1)) and np.allclose(Gd, np.swapaxes(Gd, 2, 3))
    assert np.allclose(Gd, np.conj(np.transpose(Gd, (2, 3, 0, 1, 4))))
    assert np.allclose(Gnd, np.transpose(Gnd, (2, 3, 0, 1, 4)))
    # Gamma form of the update equals the G form (eqs. Lippmann_Schwinger_strain_2/3)
    r = rng.standard_normal((3, 32)) + 1j * rng.standard_normal((3, 32))
    sig1 = rng.standard_normal((3, 3, 32)) + 1j * rng.standard_normal((3, 3, 32))
    sig1 = sig1 + np.swapaxes(sig1, 0, 1)
    sig2 = rng.standard_normal((3, 3, 32)) + 1j * rng.standard_normal((3, 3, 32))
    sig2 = sig2 + np.swapaxes(sig2, 0, 1)
    r = tetra.dot_vec(sig1, np.conj(D)) - tetra.dot_vec(sig2, D)
    g_form = np.einsum("ijkl...,kl...->ij...", Gd, sig1) + np.einsum("ijkl...,kl...->ij...", Gnd, sig2)
    gam_form = np.einsum("ijk...,k...->ij...", Gam, r)
    assert np.max(np.abs(g_form - gam_form)) < 1e-12

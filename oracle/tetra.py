"""Algorithm 1 of the paper in its own Fourier form, FP64 (test infrastructure only).

Array convention: real fields are indexed [..., l3, l2, l1] (x fastest) and
spectra [..., h3, h2, h1], with h_i = 0..N_i-1 exactly as in eq. q-vectors.
Tensors are stored as full 3x3 (or 3x3x3x3) arrays so each formula can be
read against the paper index by index.  No blocking, fusion or reordering
beyond what the equations state.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from . import voigt

WORKERS = int(os.environ.get("HZ_ORACLE_WORKERS", os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Sec. 2.2: q-grid and transforms
# ---------------------------------------------------------------------------
def qvectors(shape):
    """q_i = 2 pi h_i / N_i with h_i = 0..N_i-1 (eq. q-vectors).

    shape = (N1, N2, N3); returns q1, q2, q3 broadcastable to [N3, N2, N1]."""
    N1, N2, N3 = shape
    q1 = (2 * np.pi * np.arange(N1) / N1)[None, None, :]
    q2 = (2 * np.pi * np.arange(N2) / N2)[None, :, None]
    q3 = (2 * np.pi * np.arange(N3) / N3)[:, None, None]
    return q1, q2, q3


def FT(a):
    """Forward transform on the SC grid, A(q) = (1/N) sum_r A(r) exp(-i q.r) (eqs. FT, FT_u)."""
    n = a.shape[-1] * a.shape[-2] * a.shape[-3]
    return sfft.fftn(a, axes=(-3, -2, -1), workers=WORKERS) / n


def FTinv(a):
    """Inverse transform, A(r) = sum_q A(q) exp(i q.r), unnormalised (eqs. IFT_1, IFT_u)."""
    n = a.shape[-1] * a.shape[-2] * a.shape[-3]
    return sfft.ifftn(a, axes=(-3, -2, -1), workers=WORKERS) * n


# ---------------------------------------------------------------------------
# Sec. 2.2: Fourier symbols of the tetrahedral operators
# ---------------------------------------------------------------------------
def D_symbol(shape):
    """D_i(q) of eq. Dq on the grid of eq. q-vectors.  Shape (3, N3, N2, N1)."""
    return D_at(*qvectors(shape))


def D_at(q1, q2, q3):
    """D_i(q) of eq. Dq at arbitrary q; each term reads exp(i/2 (+-q1 +-q2 +-q3))."""
    q1, q2, q3 = np.broadcast_arrays(q1, q2, q3)
    e_ppp = np.exp(0.5j * (q1 + q2 + q3))
    e_pmm = np.exp(0.5j * (q1 - q2 - q3))
    e_mpm = np.exp(0.5j * (-q1 + q2 - q3))
    e_mmp = np.exp(0.5j * (-q1 - q2 + q3))
    D1 = 0.5 * (e_ppp + e_pmm - e_mpm - e_mmp)
    D2 = 0.5 * (e_ppp - e_pmm + e_mpm - e_mmp)
    D3 = 0.5 * (e_ppp - e_pmm - e_mpm + e_mmp)
    return np.stack([D1, D2, D3])


def singular_mask(shape):
    """True at h = (0,0,0) and h = (N1/2, N2/2, N3/2): the two modes where D vanishes
    and the Green operator is set to zero (Sec. 2.3-2.4).  Selected by integer index."""
    N1, N2, N3 = shape
    m = np.zeros((N3, N2, N1), dtype=bool)
    m[0, 0, 0] = True
    m[N3 // 2, N2 // 2, N1 // 2] = True
    return m


def green_inverse(D, C0t):
    """Omega(q)^-1 = conj(D).lambda0.D + D.lambda0.conj(D) (eq. Green_tensor):
    K_il = sum_jk lambda0_ijkl (conj(D_j) D_k + D_j conj(D_k)).  Real symmetric 3x3 per q."""
    K = np.einsum("ijkl,j...,k...->il...", C0t, np.conj(D), D, optimize=True)
    K = K + np.einsum("ijkl,j...,k...->il...", C0t, D, np.conj(D), optimize=True)
    return K


def green(D, C0t, shape):
    """Omega(q) = K(q)^-1, and Omega := 0 at the two singular modes (Sec. 2.4)."""
    K = green_inverse(D, C0t)
    Kr = np.real(K)
    assert np.max(np.abs(np.imag(K))) <= 1e-12 * max(1.0, np.max(np.abs(Kr)))
    mask = singular_mask(shape)
    Km = np.moveaxis(Kr, (0, 1), (-2, -1)).copy()
    Km[mask] = np.eye(3)
    Om = np.linalg.inv(Km)
    Om[mask] = 0.0
    return np.moveaxis(Om, (-2, -1), (0, 1))


def sym_outer(a, u):
    """(a (x)_s u)_ij = (a_i u_j + a_j u_i)/2."""
    return 0.5 * (np.einsum("i...,j...->ij...", a, u) + np.einsum("j...,i...->ij...", a, u))


def dot_vec(s, a):
    """(s . a)_i = sum_j s_ij a_j for a symmetric tensor field s."""
    return np.einsum("ij...,j...->i...", s, a)


def strain_green(D, Om):
    """G^d, G^nd (eq. strain_based_Green_functions_tetrahedral_stencil) and the
    third-order Gamma_ijk = (D_i Om_jk + D_j Om_ik)/2 (eq. Lippmann_Schwinger_strain_3)."""
    Dc = np.conj(D)

    def four(A, B):
        t = np.einsum("i...,jk...,l...->ijkl...", A, Om, B)
        return 0.25 * (t + np.swapaxes(t, 0, 1) + np.swapaxes(t, 2, 3)
                       + np.swapaxes(np.swapaxes(t, 0, 1), 2, 3))

    # four(A,B)_ijkl = 1/4 {A_i Om_jk B_l + A_j Om_ik B_l + A_i Om_jl B_k + A_j Om_il B_k}
    Gd = four(D, Dc)
    Gnd = -four(D, D)
    Gam = 0.5 * (np.einsum("i...,jk...->ijk...", D, Om) + np.einsum("j...,ik...->ijk...", D, Om))
    return Gd, Gnd, Gam


# ---------------------------------------------------------------------------
# Sec. 2.6: Algorithm 1
# ---------------------------------------------------------------------------
def _phase_indices(phase, n_phases):
    flat = phase.ravel()
    return [np.nonzero(flat == p)[0] for p in range(n_phases)]


def constitutive(eps, phase_idx, Ct, eps0t=None):
    """sigma(r) = lambda(r):(eps(r) - eps0(r)) (eq. linear_elasticity), phase by phase."""
    shp = eps.shape
    e = eps.reshape(3, 3, -1)
    s = np.zeros_like(e)
    for p, idx in enumerate(phase_idx):
        if idx.size == 0:
            continue
        ep = e[:, :, idx]
        if eps0t is not None:
            ep = ep - eps0t[p][:, :, None]
        s[:, :, idx] = np.einsum("ijkl,kln->ijn", Ct[p], ep, optimize=True)
    return s.reshape(shp)


class Result(dict):
    """Plain dict with attribute access."""

    __getattr__ = dict.__getitem__


def basic_scheme(phase, C, C0, E, tol=1e-8, max_iters=1000, eps0=None, fixed_iters=None,
                 keep_fields=True, keep_spectra=False, stress=False):
    """Displacement-based basic scheme for the tetrahedral stencil (Algorithm 1).

    phase : [N3, N2, N1] integer phase map; C : [P, 6, 6] Voigt stiffness per phase;
    C0 : [6, 6] reference medium; E : applied mean strain, tensor comps (11,22,33,23,13,12);
    eps0 : optional [P, 6] eigenstrain per phase (tensor comps).
    stress=True: E is the applied stress sigma^a instead (Sec. 2.5); the mean strain
    starts at lambda0^-1:sigma^a and follows step 6 of Algorithm 1 after every update.

    Iterate k = 0, 1, ...: build the fields of u_k, measure eps_k = L2/||<sigma>||
    (eqs. L2-norm, tolerance), stop at the first k with eps_k < tol (or at k =
    fixed_iters when given), otherwise apply the update of eq. basic_scheme_dep_2.
    The reported iterate is u_k, i.e. `iters` updates were applied.  Under applied
    stress eps_k = L2/s with the fixed scale s = ||sigma^a|| (||<lambda:eps0>|| when
    sigma^a = 0), and the stop also needs ||<sigma>_k - sigma^a|| <= tol s (the loop
    on the mean strain has converged too)."""
    phase = np.asarray(phase)
    N3, N2, N1 = phase.shape
    shape = (N1, N2, N3)
    Ct = np.stack([voigt.stiffness_tensor(c) for c in C])
    C0t = voigt.stiffness_tensor(C0)
    e0t = None if eps0 is None else np.stack([voigt.sym_tensor(e) for e in eps0])
    pidx = _phase_indices(phase, len(C))
    if stress:
        Sa = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
        Eb = voigt.solve_stiffness(C0, Sa)  # initial guess lambda0^-1 : sigma^a
        frac = np.array([idx.size for idx in pidx], dtype=np.float64) / phase.size
        C_mean = np.einsum("p,pijkl->ijkl", frac, Ct)  # <lambda>
        Ce0_mean = (np.zeros((3, 3)) if e0t is None
                    else np.einsum("p,pijkl,pkl->ij", frac, Ct, e0t))  # <lambda:eps0>
        # stress scale of the stop rule: the target ||sigma^a||, or the eigenstress
        # ||<lambda:eps0>|| when no stress is applied (<sigma> then tends to zero)
        s_ref = voigt.frobenius(Sa) or voigt.frobenius(Ce0_mean) or 1.0
    else:
        Eb = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
    Eb_hist = []

    D = D_symbol(shape)
    Om = green(D, C0t, shape)
    u = np.zeros((3, N3, N2, N1), dtype=np.complex128)  # initial guess u(q) = 0

    hist, means = [], []
    k = 0
    while True:
        # step 1: strain spectra of the two tetrahedra (eqs. desp_T1_dep_Q, desp_T2_dep_Q)
        de1q = sym_outer(D, u)
        de2q = sym_outer(-np.conj(D), u)
        # step 2: back to real space
        de1 = FTinv(de1q)
        de2 = FTinv(de2q)
        imag = max(np.max(np.abs(de1.imag)), np.max(np.abs(de2.imag)))
        de1, de2 = de1.real, de2.real
        # step 3: stresses sigma^Tk = lambda:(Ebar + deps^Tk - eps0)
        eps1 = Eb[:, :, None, None, None] + de1
        eps2 = Eb[:, :, None, None, None] + de2
        s1 = constitutive(eps1, pidx, Ct, e0t)
        s2 = constitutive(eps2, pidx, Ct, e0t)
        # step 4: forward transforms
        s1q = FT(s1)
        s2q = FT(s2)
        # equilibrium residual r(q) = sigma^T1.conj(D) - sigma^T2.D (eq. Equilibrium_Q_div_bis)
        r = dot_vec(s1q, np.conj(D)) - dot_vec(s2q, D)
        L2 = float(np.sqrt(np.sum(np.abs(r / 2) ** 2)))
        mean_sigma = 0.5 * (s1.mean(axis=(-3, -2, -1)) + s2.mean(axis=(-3, -2, -1)))
        nrm = s_ref if stress else voigt.frobenius(mean_sigma)
        err = L2 / nrm if nrm > 0 else L2
        hist.append(err)
        means.append(voigt.sym_vector(mean_sigma))
        Eb_hist.append(voigt.sym_vector(Eb))
        conv = err < tol
        if stress:
            conv = conv and voigt.frobenius(mean_sigma - Sa) <= tol * s_ref
        done = conv if fixed_iters is None else k >= fixed_iters
        if done or k >= max_iters:
            break
        # step 5: u <- u - Omega.r
        u = u - np.einsum("il...,l...->i...", Om, r)
        if stress:
            # step 6: Ebar <- lambda0^-1 : {sigma^a + (lambda0 - <lambda>):Ebar - <lambda:deps> + <lambda:eps0>}
            deps = 0.5 * (de1 + de2)
            C_deps = constitutive(deps, pidx, Ct).mean(axis=(-3, -2, -1))
            rhs = Sa + np.einsum("ijkl,kl->ij", C0t - C_mean, Eb) - C_deps + Ce0_mean
            Eb = voigt.solve_stiffness(C0, rhs)
        k += 1

    out = Result(iters=k, converged=bool(conv), residual=err, history=np.array(hist),
                 mean_sigma=voigt.sym_vector(mean_sigma), mean_history=np.array(means),
                 L2=L2, max_imag=float(imag), u_hat=u, Ebar=voigt.sym_vector(Eb),
                 Ebar_history=np.array(Eb_hist))
    if keep_fields:
        # final fields are the T1/T2 averages (eq. final_fields)
        out["eps"] = voigt.sym_vector(0.5 * (eps1 + eps2))
        out["sigma"] = voigt.sym_vector(0.5 * (s1 + s2))
        out["sigma_T1"] = s1
        out["sigma_T2"] = s2
        out["deps_T1"] = de1
        out["deps_T2"] = de2
    if keep_spectra:
        out["r_hat"] = r
        out["D"] = D
        out["Omega"] = Om
    return out


def effective_stiffness(phase, C, C0, tol=1e-8, max_iters=1000, fixed_iters=None):
    """C_eff column J = Voigt(<sigma>) for the unit load gamma_J = 1 (Sec. 2.6 final fields)."""
    cols, infos = [], []
    for J in range(6):
        E = np.zeros(6)
        E[J] = 1.0 if J < 3 else 0.5
        res = basic_scheme(phase, C, C0, E, tol=tol, max_iters=max_iters,
                           fixed_iters=fixed_iters, keep_fields=False)
        cols.append(res.mean_sigma)
        infos.append(res)
    return np.array(cols).T, infos


# ---------------------------------------------------------------------------
# Sec. 2.6: Algorithm 2 (strain-based form), used to check Algorithm 1 step by step
# ---------------------------------------------------------------------------
def strain_scheme(phase, C, C0, E, n_iters):
    """Algorithm 2 with the Gamma update of eq. Lippmann_Schwinger_strain_3, run for
    n_iters updates from deps = 0; returns the history of eps_k and <sigma>_k."""
    phase = np.asarray(phase)
    N3, N2, N1 = phase.shape
    shape = (N1, N2, N3)
    Ct = np.stack([voigt.stiffness_tensor(c) for c in C])
    C0t = voigt.stiffness_tensor(C0)
    Eb = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
    pidx = _phase_indices(phase, len(C))
    D = D_symbol(shape)
    Om = green(D, C0t, shape)
    _, _, Gam = strain_green(D, Om)
    de1q = np.zeros((3, 3, N3, N2, N1), dtype=np.complex128)
    de2q = np.zeros_like(de1q)
    hist, means = [], []
    for k in range(n_iters + 1):
        de1 = FTinv(de1q).real
        de2 = FTinv(de2q).real
        s1 = constitutive(Eb[:, :, None, None, None] + de1, pidx, Ct)
        s2 = constitutive(Eb[:, :, None, None, None] + de2, pidx, Ct)
        s1q, s2q = FT(s1), FT(s2)
        r = dot_vec(s1q, np.conj(D)) - dot_vec(s2q, D)
        mean_sigma = 0.5 * (s1.mean(axis=(-3, -2, -1)) + s2.mean(axis=(-3, -2, -1)))
        hist.append(float(np.sqrt(np.sum(np.abs(r / 2) ** 2))) / voigt.frobenius(mean_sigma))
        means.append(voigt.sym_vector(mean_sigma))
        if k == n_iters:
            break
        de1q = de1q - np.einsum("ijk...,k...->ij...", Gam, r)
        de2q = de2q + np.einsum("ijk...,k...->ij...", np.conj(Gam), r)
    return np.array(hist), np.array(means)

"""Comparison Green operators of the paper's experiments, FP64 (test infrastructure only).

Sec. 3.2 and Appendix B compare the tetrahedral scheme with two other
discretisations of the same displacement-based basic scheme, each with ONE
strain field per voxel, eps = Ebar + D(q) (x)_s u(q):

* the rotated scheme (Willot): D(q) of eq. Dq_rotated, the 8-corner finite
  differences of a staggered displacement grid;
* the continuous-frequency operator of Moulinec-Suquet: D(q) = i xi(q) with xi
  the frequency of the centred representative of q.

Both use the displacement Lippmann-Schwinger form of Appendix B (eq.
displacement_Lippmann_Schwinger_rotated): Omega(q)^-1 = conj(D).lambda0.D
(eq. inverse_displacement_Green_function_rotated), the equilibrium residual
r(q) = sigma(q).conj(D(q)) and the update u <- u - Omega.r.  Where D vanishes
away from q = 0 the Green function is undefined; Willot's recipe quoted in
Sec. 3.2 sets it to zero there.  The continuous operator's treatment of the
highest frequency of an even axis is a reading (stated at continuous_symbol).

Array conventions as in ``tetra``: real fields [..., l3, l2, l1], spectra
[..., h3, h2, h1] with h_i = 0..N_i-1.  Plain and unblocked, to be read
against the equations.
"""
from __future__ import annotations

import numpy as np

from . import tetra, voigt


def rotated_symbol(shape):
    """D_i(q) of the rotated scheme (eq. Dq_rotated): D_i = 1/4 (e^{iq_i} - 1) times
    (e^{iq_j} + 1) for the two other axes j.  Shape (3, N3, N2, N1)."""
    q1, q2, q3 = tetra.qvectors(shape)
    m = [np.exp(1j * q) - 1.0 for q in (q1, q2, q3)]
    p = [np.exp(1j * q) + 1.0 for q in (q1, q2, q3)]
    D1 = 0.25 * m[0] * p[1] * p[2]
    D2 = 0.25 * p[0] * m[1] * p[2]
    D3 = 0.25 * p[0] * p[1] * m[2]
    return np.stack(np.broadcast_arrays(D1, D2, D3))


def rotated_singular(shape):
    """Where D of eq. Dq_rotated vanishes: q = 0, and every q with at least two
    components equal to pi (only on even axes; Appendix B).  By integer index."""
    N1, N2, N3 = shape
    h1 = np.arange(N1)[None, None, :]
    h2 = np.arange(N2)[None, :, None]
    h3 = np.arange(N3)[:, None, None]
    at_pi = (2 * h1 == N1).astype(int) + (2 * h2 == N2).astype(int) + (2 * h3 == N3).astype(int)
    zero = (h1 == 0) & (h2 == 0) & (h3 == 0)
    return zero | (at_pi >= 2)


def centred_frequency(N):
    """xi(h) = 2 pi h~ / N with h~ the representative of h in (-N/2, N/2); the highest
    frequency h = N/2 of an even N is given xi = 0 (see continuous_symbol)."""
    h = np.arange(N)
    ht = np.where(2 * h < N, h, h - N).astype(np.float64)
    ht[2 * h == N] = 0.0
    return 2 * np.pi * ht / N


def continuous_symbol(shape):
    """D(q) = i xi(q) of the continuous-frequency (Moulinec-Suquet) operator.

    Reading: on an even axis the frequency q = pi has two representatives, +pi and
    -pi, and i xi cannot satisfy D(-q) = conj(D(q)) there, which Sec. 3.2 notes
    makes the back-transformed strain complex.  The paper's runs fix the strain
    Green function to lambda0^-1 at those points (Moulinec-Suquet's recipe for the
    strain-based scheme), which has no counterpart in the displacement form used
    here; this oracle takes the symmetric derivative instead: xi = 0 at h = N/2
    (the derivative of the band-limited interpolant whose highest mode is a
    cosine), so the strain stays real and is a gradient at every q."""
    N1, N2, N3 = shape
    x1 = centred_frequency(N1)[None, None, :]
    x2 = centred_frequency(N2)[None, :, None]
    x3 = centred_frequency(N3)[:, None, None]
    return 1j * np.stack(np.broadcast_arrays(x1, x2, x3)).astype(np.complex128)


def continuous_singular(shape):
    """Where i xi vanishes: every h_a in {0, N_a/2}.  By integer index."""
    N1, N2, N3 = shape
    m1 = (np.arange(N1) == 0) | (2 * np.arange(N1) == N1)
    m2 = (np.arange(N2) == 0) | (2 * np.arange(N2) == N2)
    m3 = (np.arange(N3) == 0) | (2 * np.arange(N3) == N3)
    return m3[:, None, None] & m2[None, :, None] & m1[None, None, :]


OPERATORS = {
    "rotated": (rotated_symbol, rotated_singular),
    "continuous": (continuous_symbol, continuous_singular),
}


def green(D, C0t, mask):
    """Omega(q) = (conj(D).lambda0.D)^-1 (eq. inverse_displacement_Green_function_rotated),
    Omega := 0 on the mask (Willot's recipe).  K_ik = sum_jl conj(D_j) lambda0_jikl D_l."""
    K = np.einsum("jikl,j...,l...->ik...", C0t, np.conj(D), D, optimize=True)
    Kr = np.real(K)
    assert np.max(np.abs(np.imag(K))) <= 1e-12 * max(1.0, np.max(np.abs(Kr)))
    Km = np.moveaxis(Kr, (0, 1), (-2, -1)).copy()
    Km[mask] = np.eye(3)
    Om = np.linalg.inv(Km)
    Om[mask] = 0.0
    return np.moveaxis(Om, (-2, -1), (0, 1))


def basic_scheme(phase, C, C0, E, operator, tol=1e-8, max_iters=1000, eps0=None, fixed_iters=None,
                 stress=False):
    """The displacement-based basic scheme with one strain field per voxel and the
    gradient symbol of `operator` ("rotated" or "continuous").

    Iterate k = 0, 1, ...: eps_k = Ebar + FT^-1[D (x)_s u_k], sigma_k = lambda:(eps_k - eps0),
    r_k = FT[sigma_k].conj(D), eps_k^err = sqrt(sum_q |r_k|^2)/||<sigma_k>|| (the measure of
    eq. tolerance for a single strain field), stop at the first k below tol (or at
    k = fixed_iters), else u <- u - Omega.r.  stress=True: E is the applied stress and
    the mean strain follows step 6 of Algorithm 1 after every update, with the stop
    rule of the tetrahedral oracle (fixed scale ||sigma^a||, mean stress at target)."""
    sym_fn, mask_fn = OPERATORS[operator]
    phase = np.asarray(phase)
    N3, N2, N1 = phase.shape
    shape = (N1, N2, N3)
    Ct = np.stack([voigt.stiffness_tensor(c) for c in C])
    C0t = voigt.stiffness_tensor(C0)
    e0t = None if eps0 is None else np.stack([voigt.sym_tensor(e) for e in eps0])
    pidx = tetra._phase_indices(phase, len(C))
    if stress:
        Sa = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
        Eb = voigt.solve_stiffness(C0, Sa)
        frac = np.array([idx.size for idx in pidx], dtype=np.float64) / phase.size
        C_mean = np.einsum("p,pijkl->ijkl", frac, Ct)
        Ce0_mean = (np.zeros((3, 3)) if e0t is None
                    else np.einsum("p,pijkl,pkl->ij", frac, Ct, e0t))
        s_ref = voigt.frobenius(Sa) or voigt.frobenius(Ce0_mean) or 1.0
    else:
        Eb = voigt.sym_tensor(np.asarray(E, dtype=np.float64))

    D = sym_fn(shape)
    Om = green(D, C0t, mask_fn(shape))
    u = np.zeros((3, N3, N2, N1), dtype=np.complex128)
    hist, means, Eb_hist = [], [], []
    k = 0
    while True:
        de = tetra.FTinv(tetra.sym_outer(D, u))
        imag = float(np.max(np.abs(de.imag)))
        de = de.real
        eps = Eb[:, :, None, None, None] + de
        s = tetra.constitutive(eps, pidx, Ct, e0t)
        r = tetra.dot_vec(tetra.FT(s), np.conj(D))
        L2 = float(np.sqrt(np.sum(np.abs(r) ** 2)))
        mean_sigma = s.mean(axis=(-3, -2, -1))
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
        u = u - np.einsum("il...,l...->i...", Om, r)
        if stress:
            C_deps = tetra.constitutive(de, pidx, Ct).mean(axis=(-3, -2, -1))
            rhs = Sa + np.einsum("ijkl,kl->ij", C0t - C_mean, Eb) - C_deps + Ce0_mean
            Eb = voigt.solve_stiffness(C0, rhs)
        k += 1
    return tetra.Result(iters=k, converged=bool(conv), residual=err, history=np.array(hist),
                        mean_sigma=voigt.sym_vector(mean_sigma), mean_history=np.array(means),
                        max_imag=imag, u_hat=u, D=D, Omega=Om, Ebar=voigt.sym_vector(Eb),
                        Ebar_history=np.array(Eb_hist), eps=voigt.sym_vector(eps),
                        sigma=voigt.sym_vector(s))

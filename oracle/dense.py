"""Plain definition of the discrete problem on tiny grids (test infrastructure only).

The collapsed energy E = 1/2 (E^(1) + E^(2)) of eqs. Elast_energy_k and
Elast_energy is, with d = 1 and the T1/T2 bookkeeping of eq. X_T1_T2_R,

    E(U) = 1/4 sum_r sum_{k=1,2} (Ebar + B_k U - eps0)(r) : lambda(r) : (Ebar + B_k U - eps0)(r)

where U collects the corner displacements and B_k is the tetrahedral
gradient of eqs. deps, DA1-DA2.  Mechanical equilibrium (eq. Equilibrium_real)
is dE/dU = 0, a symmetric positive semi-definite linear system whose null
space holds the uniform translations of each FCC corner subgrid.  It is
assembled densely and solved by least squares.  Used only for N <= a few
hundred voxels.
"""
import numpy as np

from . import voigt
from .stencil import T1_OFFSETS, T2_OFFSETS


def gradient_matrix(shape, tet):
    """B_k: (9N x 3N) real matrix, strain component (i,j) at voxel r from corner displacements."""
    N1, N2, N3 = shape
    n = N1 * N2 * N3
    offs = T1_OFFSETS if tet == 1 else T2_OFFSETS
    B = np.zeros((3, 3, n, 3, n))

    def vid(l1, l2, l3):
        return (l3 % N3) * N2 * N1 + (l2 % N2) * N1 + (l1 % N1)

    for l3 in range(N3):
        for l2 in range(N2):
            for l1 in range(N1):
                r = vid(l1, l2, l3)
                for v in offs:
                    o = (v - 0.5).astype(int)
                    c = vid(l1 + o[0], l2 + o[1], l3 + o[2])
                    for i in range(3):
                        for j in range(3):
                            B[i, j, r, j, c] += 0.5 * v[i]
                            B[i, j, r, i, c] += 0.5 * v[j]
    return B.reshape(9 * n, 3 * n)


def minimise(phase, C, E, eps0=None, stress=False):
    """Equilibrium by direct minimisation of E(U).  Returns dict with mean stress
    (tensor comps), the T1/T2 strain and stress fields, and the null-space dimension.

    stress=True: E is an applied stress sigma^a and the mean strain Ebar joins the
    unknowns; the functional gains the external work -N sigma^a:Ebar
    (eq. Grand_Elast_energy, d = 1), whose stationarity in Ebar is <sigma> = sigma^a."""
    phase = np.asarray(phase)
    N3, N2, N1 = phase.shape
    shape = (N1, N2, N3)
    n = N1 * N2 * N3
    Ct = np.stack([voigt.stiffness_tensor(c) for c in C])
    Cvox = Ct[phase.ravel()]  # [n,3,3,3,3]
    # block-diagonal material operator on 9N strain vectors (component-major)
    L = np.zeros((3, 3, n, 3, 3, n))
    idx = np.arange(n)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    L[i, j, idx, k, l, idx] = Cvox[:, i, j, k, l]
    L = L.reshape(9 * n, 9 * n)
    Bs = [gradient_matrix(shape, 1), gradient_matrix(shape, 2)]
    e0f = np.zeros(9 * n)
    if eps0 is not None:
        e0 = np.stack([voigt.sym_tensor(e) for e in eps0])[phase.ravel()]  # [n,3,3]
        e0f = np.moveaxis(e0, 0, -1).reshape(9 * n)
    A = sum(B.T @ L @ B for B in Bs)
    if stress:
        # P: the six independent components of Ebar -> the uniform 9N strain field
        P = np.zeros((9, n, 6))
        for m, (i, j) in enumerate(voigt.PAIRS):
            P[i * 3 + j, :, m] = 1.0
            P[j * 3 + i, :, m] = 1.0
        P = P.reshape(9 * n, 6)
        Sa = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
        work = P.T @ np.repeat(Sa.reshape(9, 1), n, axis=1).reshape(9 * n)  # d(sigma^a:Ebar)/de_m per voxel, summed
        # dE/dU = 1/2 sum_k B_k^T L (P e + B_k U - e0) = 0
        # dE/de = 1/2 sum_k P^T L (P e + B_k U - e0) - N sigma^a:dEbar/de = 0
        BLP = sum(B.T @ L @ P for B in Bs)
        K = np.block([[A, BLP], [BLP.T, 2.0 * P.T @ L @ P]])
        rhs = np.concatenate([sum(B.T @ L @ e0f for B in Bs),
                              2.0 * P.T @ L @ e0f + 2.0 * work])
        x, *_ = np.linalg.lstsq(K, rhs, rcond=None)
        U, e = x[:3 * n], x[3 * n:]
        Eb = (P.reshape(9, n, 6)[:, 0, :] @ e).reshape(3, 3)
    else:
        Eb = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
        b = -sum(B.T @ L @ (np.repeat(Eb.reshape(9, 1), n, axis=1).reshape(9 * n) - e0f)
                 for B in Bs)
        U, *_ = np.linalg.lstsq(A, b, rcond=None)
    e_bar = np.repeat(Eb.reshape(9, 1), n, axis=1).reshape(9 * n) - e0f
    w = np.linalg.eigvalsh(A)
    null_dim = int(np.sum(np.abs(w) <= 1e-10 * np.max(np.abs(w))))
    out = {"U": U, "null_dim": null_dim, "Ebar": voigt.sym_vector(Eb)}
    sig = []
    for k, B in enumerate(Bs, start=1):
        eps = (Eb.reshape(9, 1) + (B @ U).reshape(9, n)).reshape(3, 3, N3, N2, N1)
        s = (L @ (e_bar + B @ U)).reshape(3, 3, N3, N2, N1)
        out[f"eps_T{k}"] = eps
        out[f"sigma_T{k}"] = s
        sig.append(s)
    ms = 0.5 * (sig[0].mean(axis=(-3, -2, -1)) + sig[1].mean(axis=(-3, -2, -1)))
    out["mean_sigma"] = voigt.sym_vector(ms)
    out["energy"] = 0.25 * sum(
        float((e_bar + B @ U) @ L @ (e_bar + B @ U)) for B in Bs)
    return out

"""Real-space tetrahedral finite-difference operators (eqs. DA1-DA2) and the corner
force density of eq. L2-norm (test infrastructure only).

Displacements live on the SC corner grid.  Corner arrays are indexed by an
integer c = (c1, c2, c3) standing for the site at position c + (1/2, 1/2, 1/2);
voxel r has the eight corners r + o, o in {0,-1}^3, at offset v = o + (1/2,1/2,1/2).

Eq. DA1: the scheme-1 operator on A sites uses the four corners
r + (111)/2, r + (1-1-1)/2, r + (-1-11)/2, r + (-11-1)/2 with weight v_i
(each term carries 1/2 and the sign of the i-th offset).  Eq. DB2 gives the
same operator on B sites, so the tetrahedron "T1" (eq. X_T1_T2_R) uses these
four corners at every voxel.  Eqs. DB1/DA2 apply the central symmetry with a
minus sign, so "T2" uses the four opposite corners, again with weight v_i.
"""
import numpy as np

T1_OFFSETS = [np.array(v) / 2 for v in ((1, 1, 1), (1, -1, -1), (-1, -1, 1), (-1, 1, -1))]
T2_OFFSETS = [-v for v in T1_OFFSETS]


def _corner_shift(u, v):
    """Sample corner field u at r + v for every voxel r (periodic); v in {+-1/2}^3.

    Corner index c = r + v - 1/2, so the sample is u[c] with c_a = r_a + o_a,
    o = v - 1/2 in {0, -1}; arrays are [.., l3, l2, l1]."""
    o = (v - 0.5).astype(int)  # (o1, o2, o3)
    return np.roll(u, shift=(-o[2], -o[1], -o[0]), axis=(-3, -2, -1))


def grad(u, tet):
    """Fluctuating strain of one tetrahedron: eps_ij(r) = 1/2 (D_i[u_j] + D_j[u_i])(r)
    with D_i[f](r) = sum_v v_i f(r+v) (eqs. deps, DA1-DA2).  u: [3, N3, N2, N1] on corners."""
    offs = T1_OFFSETS if tet == 1 else T2_OFFSETS
    g = np.zeros((3, 3) + u.shape[1:])
    for v in offs:
        us = _corner_shift(u, v)
        for i in range(3):
            for j in range(3):
                g[i, j] += v[i] * us[j]
    return 0.5 * (g + np.swapaxes(g, 0, 1))


def force(s1, s2):
    """Corner force density f(c) = dE/du(c) for E = 1/2 (E^(1)+E^(2)) (eqs. Elast_energy_k,
    Elast_energy), d = 1: f_i(c) = 1/2 [ sum_{v in T1} sigma^T1_ij(c - v) v_j
                                        + sum_{v in T2} sigma^T2_ij(c - v) v_j ]."""
    f = np.zeros((3,) + s1.shape[2:])
    for offs, s in ((T1_OFFSETS, s1), (T2_OFFSETS, s2)):
        for v in offs:
            o = (v - 0.5).astype(int)
            # voxel r = c - o feeds corner c; roll brings s(c - o) to index c
            ss = np.roll(s, shift=(o[2], o[1], o[0]), axis=(-3, -2, -1))
            for i in range(3):
                for j in range(3):
                    f[i] += 0.5 * v[j] * ss[i, j]
    return f


def corner_FT(f):
    """(1/N) sum_c f(c) exp(-i q.(c + 1/2)) over corner positions (eq. FT_u), h_i = 0..N_i-1."""
    N3, N2, N1 = f.shape[-3:]
    n = N1 * N2 * N3
    F = np.fft.fftn(f, axes=(-3, -2, -1)) / n
    q1 = 2 * np.pi * np.arange(N1) / N1
    q2 = 2 * np.pi * np.arange(N2) / N2
    q3 = 2 * np.pi * np.arange(N3) / N3
    ph = np.exp(-0.5j * (q1[None, None, :] + q2[None, :, None] + q3[:, None, None]))
    return F * ph

"""Seeded synthetic inputs for the tetrahedral-stencil FFT homogenization solver.

This module prepares *inputs only*: voxel phase maps, per-phase stiffness
tables (6x6 engineering-shear Voigt, order 11,22,33,23,13,12), macroscopic
load cases and the reference-medium choices the paper uses in its
experiments.  It holds none of the solver's arithmetic (no Fourier symbols,
no Green operator, no iteration) and is the only code shared between the
CPU oracle and the HIP path.

Geometry conventions: voxel (l1, l2, l3) has its centre at integer
coordinates (Sec. 2.1, eq. r-vectors); phase maps are numpy arrays indexed
``phase[l3, l2, l1]`` (x fastest in memory), dtype uint16.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


# --------------------------------------------------------------------------
# materials
# --------------------------------------------------------------------------
def isotropic_voigt(E: float, nu: float) -> np.ndarray:
    """6x6 engineering-shear Voigt stiffness of an isotropic solid (E, nu).

    E = 0 gives the all-zero stiffness of a void (Sec. 3.2)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for i in range(3):
        C[i, i] = lam + 2.0 * mu
        C[3 + i, 3 + i] = mu
    return C


def cubic_voigt(C11: float, C12: float, C44: float) -> np.ndarray:
    """6x6 Voigt stiffness of a cubic crystal in its own frame."""
    C = np.zeros((6, 6))
    C[:3, :3] = C12
    for i in range(3):
        C[i, i] = C11
        C[3 + i, 3 + i] = C44
    return C


def _voigt_to_tensor(C: np.ndarray) -> np.ndarray:
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            v = C[I, J]
            T[i, j, k, l] = T[j, i, k, l] = T[i, j, l, k] = T[j, i, l, k] = v
    return T


def _tensor_to_voigt(T: np.ndarray) -> np.ndarray:
    C = np.zeros((6, 6))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            C[I, J] = T[i, j, k, l]
    return C


def rotate_voigt(C: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Stiffness of a crystal whose frame is rotated by R: C'_ijkl = R_ia R_jb R_kc R_ld C_abcd."""
    T = _voigt_to_tensor(C)
    Tr = np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, T, optimize=True)
    return _tensor_to_voigt(Tr)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices uniform on SO(3) via uniform unit quaternions (Shoemake 1992)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    z, w = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_spd_voigt(rng: np.random.Generator, lo: float, hi: float) -> np.ndarray:
    """A random triclinic (fully anisotropic) stiffness whose Mandel eigenvalues lie in [lo, hi]."""
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    ev = lo + (hi - lo) * rng.random(6)
    M = (Q * ev) @ Q.T  # Mandel form
    s = np.array([1, 1, 1, math.sqrt(2), math.sqrt(2), math.sqrt(2)])
    return M / np.outer(s, s)


def unit_load(J: int) -> np.ndarray:
    """Unit macroscopic strain of load case J as tensor components (11,22,33,23,13,12).

    Case J has engineering strain gamma_J = 1, so shear cases have eps_ij = 1/2."""
    E = np.zeros(6)
    E[J] = 1.0 if J < 3 else 0.5
    return E


# --------------------------------------------------------------------------
# reference media (the paper's per-experiment choices)
# --------------------------------------------------------------------------
def ref_alpha_rule(E_matrix: float, E_incl: float, nu: float) -> np.ndarray:
    """Isotropic reference medium of the contrast study (Sec. 3.4): same nu,
    k0 = alpha k_m + (1-alpha) k_i with alpha = 0.45 for a stiffer inclusion
    and 0.55 for a softer one (equal nu makes k proportional to E)."""
    alpha = 0.45 if E_incl > E_matrix else 0.55
    return isotropic_voigt(alpha * E_matrix + (1.0 - alpha) * E_incl, nu)


def ref_cubic_polycrystal(C11: float, C12: float, C44: float) -> np.ndarray:
    """Isotropic reference for a cubic polycrystal: bulk (C11+2C12)/3 and shear
    modulus the mean of the two cubic shear moduli (C11-C12)/2 and C44."""
    K0 = (C11 + 2.0 * C12) / 3.0
    mu0 = 0.5 * (0.5 * (C11 - C12) + C44)
    lam0 = K0 - 2.0 * mu0 / 3.0
    C = np.zeros((6, 6))
    C[:3, :3] = lam0
    for i in range(3):
        C[i, i] = lam0 + 2 * mu0
        C[3 + i, 3 + i] = mu0
    return C


# --------------------------------------------------------------------------
# microstructures
# --------------------------------------------------------------------------
def centred_sphere(n: int, target_vf: float = 0.2) -> tuple[np.ndarray, float]:
    """Phase map (0 matrix, 1 sphere) of a sphere centred in an n^3 cell.

    Centre at (n/2 - 1/2) in voxel-centre coordinates; a voxel is inside when
    |r - c|^2 <= R^2.  R^2 is the distinct squared distance whose voxel count
    is closest to target_vf * n^3 (ties: the smaller radius)."""
    c = n / 2.0 - 0.5
    l = np.arange(n) - c
    d2 = l[:, None, None] ** 2 + l[None, :, None] ** 2 + l[None, None, :] ** 2
    vals, counts = np.unique(d2, return_counts=True)
    cum = np.cumsum(counts)
    k = int(np.argmin(np.abs(cum - target_vf * n ** 3)))
    R2 = float(vals[k])
    return (d2 <= R2).astype(np.uint16), R2


def boolean_spheres(shape, radius: float, target_vf: float, seed: int):
    """Boolean model of overlapping spheres in a periodic cell.

    Centres are uniform and continuous in [0, N_i); a voxel belongs to a
    sphere when its periodic minimum-image distance to the centre is <=
    radius.  Spheres are added one at a time until the voxel volume fraction
    first reaches target_vf.  Returns (phase[l3,l2,l1] uint16, n_spheres, vf)."""
    N1, N2, N3 = shape
    rng = np.random.default_rng(seed)
    phase = np.zeros((N3, N2, N1), dtype=np.uint16)
    total = N1 * N2 * N3
    count = 0
    ns = 0
    r = int(math.ceil(radius))
    off = np.arange(-r - 1, r + 2)
    while count < target_vf * total:
        cx, cy, cz = rng.random(3) * np.array([N1, N2, N3])
        ix = np.round(cx).astype(int) + off
        iy = np.round(cy).astype(int) + off
        iz = np.round(cz).astype(int) + off
        dx = ix - cx
        dy = iy - cy
        dz = iz - cz
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        m = d2 <= radius * radius
        zz, yy, xx = np.nonzero(m)
        gz, gy, gx = iz[zz] % N3, iy[yy] % N2, ix[xx] % N1
        sub = phase[gz, gy, gx]
        count += int(np.count_nonzero(sub == 0))
        phase[gz, gy, gx] = 1
        ns += 1
    return phase, ns, count / total


def voronoi(shape, n_grains: int, seed: int):
    """Periodic Voronoi tessellation: voxel -> nearest of n_grains uniform
    continuous seeds (periodic minimum-image Euclidean distance).  Returns
    (grain id map [l3,l2,l1] uint16, rng positioned after the seed draws)."""
    from scipy.spatial import cKDTree

    N1, N2, N3 = shape
    rng = np.random.default_rng(seed)
    seeds = rng.random((n_grains, 3)) * np.array([N1, N2, N3])
    tree = cKDTree(seeds, boxsize=[N1, N2, N3])
    gz, gy, gx = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1).astype(np.float64)
    # points exactly on the upper box face are folded back by the periodic tree
    _, idx = tree.query(pts, k=1, workers=-1)
    return idx.reshape(N3, N2, N1).astype(np.uint16), rng


def laminate(shape, axis: int, n_phases: int, seed: int) -> np.ndarray:
    """Random layered microstructure: the phase depends only on the coordinate along `axis` (0=x,1=y,2=z)."""
    rng = np.random.default_rng(seed)
    n_ax = shape[axis]
    layer = rng.integers(0, n_phases, n_ax).astype(np.uint16)
    layer[: n_phases] = np.arange(n_phases)  # every phase present
    N1, N2, N3 = shape
    ph = np.empty((N3, N2, N1), dtype=np.uint16)
    if axis == 0:
        ph[:] = layer[None, None, :]
    elif axis == 1:
        ph[:] = layer[None, :, None]
    else:
        ph[:] = layer[:, None, None]
    return ph


# --------------------------------------------------------------------------
# workload recipes
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """One homogenization problem: grid, phases, stiffness table, reference medium, loads."""

    name: str
    shape: tuple
    phase: np.ndarray  # [N3, N2, N1] uint16
    C: np.ndarray  # [n_phases, 6, 6] Voigt
    C0: np.ndarray  # [6, 6] reference medium (Voigt)
    loads: np.ndarray  # [n_loads, 6] tensor components
    tol: float
    info: dict = field(default_factory=dict)


def sphere16() -> Problem:
    """16^3, centred sphere at ~20% volume fraction, matrix E=1 inclusion E=10 (nu=0.3)."""
    ph, R2 = centred_sphere(16, 0.2)
    C = np.stack([isotropic_voigt(1.0, 0.3), isotropic_voigt(10.0, 0.3)])
    C0 = ref_alpha_rule(1.0, 10.0, 0.3)
    loads = np.array([[1e-3, 0, 0, 0, 0, 0]], dtype=np.float64)
    return Problem("sphere16", (16, 16, 16), ph, C, C0, loads, 1e-8,
                   {"R2": R2, "vf": float(ph.mean())})


def boolean128(n: int = 128, contrast: float = 1e3, seed: int = 2, vf: float = 0.30,
               radius: float = 8.0) -> Problem:
    """Boolean overlapping spheres (radius 8 voxels) to 30% volume fraction in an
    n^3 cell, sphere/matrix stiffness contrast 1e3 at nu=0.3, 6 unit loads."""
    ph, ns, avf = boolean_spheres((n, n, n), radius, vf, seed)
    C = np.stack([isotropic_voigt(1.0, 0.3), isotropic_voigt(contrast, 0.3)])
    C0 = ref_alpha_rule(1.0, contrast, 0.3)
    loads = np.stack([unit_load(J) for J in range(6)])
    return Problem(f"boolean{n}_c{contrast:g}", (n, n, n), ph, C, C0, loads, 1e-8,
                   {"n_spheres": ns, "vf": avf, "seed": seed, "radius": radius})


def polycrystal(shape=(256, 256, 256), n_grains: int = 200, seed: int = 3,
                C11: float = 168.0, C12: float = 121.0, C44: float = 75.0,
                tol: float = 1e-6) -> Problem:
    """Periodic Voronoi polycrystal of cubic grains with uniform random orientations."""
    ph, rng = voronoi(shape, n_grains, seed)
    Rs = random_rotations(rng, n_grains)
    base = cubic_voigt(C11, C12, C44)
    C = np.stack([rotate_voigt(base, R) for R in Rs])
    C0 = ref_cubic_polycrystal(C11, C12, C44)
    loads = np.stack([unit_load(J) for J in range(6)])
    return Problem(f"voronoi{shape[0]}x{shape[1]}x{shape[2]}", tuple(shape), ph, C, C0, loads,
                   tol, {"n_grains": n_grains, "seed": seed})


def sphere_contrast(shape, contrast, seed: int = 4, vf: float = 0.25, radius: float = 8.0,
                    tol: float = 1e-6) -> Problem:
    """Boolean spheres to 25% in matrix E=1 (nu=0.3): contrast = E_incl/E_matrix;
    contrast 0 means voids, np.inf is mapped to 1e8 (rigid inclusions)."""
    ph, ns, avf = boolean_spheres(shape, radius, vf, seed)
    Ei = 1e8 if contrast == np.inf else float(contrast)
    C = np.stack([isotropic_voigt(1.0, 0.3), isotropic_voigt(Ei, 0.3)])
    C0 = ref_alpha_rule(1.0, Ei, 0.3)
    loads = np.array([unit_load(0)])
    return Problem(f"spheres{shape[0]}x{shape[1]}x{shape[2]}_c{contrast:g}", tuple(shape), ph,
                   C, C0, loads, tol, {"n_spheres": ns, "vf": avf})


def isolated_sphere(contrast: float, n: int = 48, radius_frac: float = 0.4, nu: float = 0.125) -> Problem:
    """The contrast study's isolated inclusion (Sec. 3.4): one sphere of radius
    radius_frac * n centred in an n^3 cell (voxel-centre coordinates, |r - c| <= R),
    matrix E = 1, inclusion E = contrast (0: a void), both with Poisson ratio nu,
    the alpha-rule reference medium, load E_xx."""
    c = n / 2.0 - 0.5
    l = np.arange(n) - c
    d2 = l[:, None, None] ** 2 + l[None, :, None] ** 2 + l[None, None, :] ** 2
    ph = (d2 <= (radius_frac * n) ** 2).astype(np.uint16)
    C = np.stack([isotropic_voigt(1.0, nu), isotropic_voigt(contrast, nu)])
    C0 = ref_alpha_rule(1.0, contrast, nu)
    return Problem(f"isolated{n}_c{contrast:g}", (n, n, n), ph, C, C0, np.array([unit_load(0)]), 1e-10,
                   {"contrast": contrast, "vf": float(ph.mean())})


def hard_sphere(n: int = 128, radius: float = 40.0) -> Problem:
    """The hard inclusion of Sec. 3.3: one glass sphere (E = 72 GPa, nu = 0.22) of radius
    40 voxels centred in a 128^3 polyamide cell (E = 2.1 GPa, nu = 0.3), moduli in MPa,
    reference medium the mean of the two stiffnesses, applied strain eps_11 = 0.05."""
    c = n / 2.0 - 0.5
    l = np.arange(n) - c
    d2 = l[:, None, None] ** 2 + l[None, :, None] ** 2 + l[None, None, :] ** 2
    ph = (d2 <= radius ** 2).astype(np.uint16)
    C = np.stack([isotropic_voigt(2.1e3, 0.3), isotropic_voigt(72.0e3, 0.22)])
    return Problem(f"hard_sphere{n}", (n, n, n), ph, C, 0.5 * (C[0] + C[1]),
                   np.array([[0.05, 0, 0, 0, 0, 0]]), 1e-10, {"vf": float(ph.mean())})


def serving_request_params(i: int, sizes=(32, 48, 64, 96, 128, 160, 192), base_seed: int = 5):
    """Grid size n, microstructure kind, contrast and load index J of request i of the
    serving stream (the draws of its generator, without building the microstructure)."""
    rng = np.random.default_rng([base_seed, i])
    n = int(rng.choice(sizes))
    kind = "spheres" if rng.random() < 0.5 else "polycrystal"
    contrast = float(10.0 ** rng.uniform(1.0, 6.0))
    J = int(rng.integers(0, 6))
    return n, kind, contrast, J


def serving_request(i: int, sizes=(32, 48, 64, 96, 128, 160, 192), base_seed: int = 5):
    """Request i of the serving stream: grid size, microstructure kind, contrast and
    load drawn from the stream's generator; the microstructure from seed 1000+i."""
    n, kind, contrast, J = serving_request_params(i, sizes, base_seed)
    seed = 1000 + i
    if kind == "spheres":
        ph, ns, avf = boolean_spheres((n, n, n), n / 16.0, 0.3, seed)
        C = np.stack([isotropic_voigt(1.0, 0.3), isotropic_voigt(contrast, 0.3)])
        C0 = ref_alpha_rule(1.0, contrast, 0.3)
    else:
        ng = 200
        ph, grng = voronoi((n, n, n), ng, seed)
        Rs = random_rotations(grng, ng)
        K = (168.0 + 2 * 121.0) / 3.0
        Cp = 0.5 * (168.0 - 121.0)
        C44 = contrast * Cp
        C11 = K + 4.0 * Cp / 3.0
        C12 = K - 2.0 * Cp / 3.0
        base = cubic_voigt(C11, C12, C44)
        C = np.stack([rotate_voigt(base, R) for R in Rs])
        C0 = ref_cubic_polycrystal(C11, C12, C44)
    return Problem(f"req{i}", (n, n, n), ph, C, C0, np.array([unit_load(J)]), 1e-6,
                   {"kind": kind, "contrast": contrast, "J": J})

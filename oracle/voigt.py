"""Voigt <-> tensor bookkeeping for the oracle (test infrastructure only).

Stiffness tables use the engineering-shear Voigt matrix, sigma_I = C_IJ gamma_J
with gamma = (e11, e22, e33, 2e23, 2e13, 2e12); strains and stresses given as
vectors use the tensor components in the order (11, 22, 33, 23, 13, 12).
"""
import numpy as np

PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def stiffness_tensor(C):
    """6x6 Voigt -> 3x3x3x3 tensor with minor and major symmetries."""
    C = np.asarray(C, dtype=np.float64)
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(PAIRS):
        for J, (k, l) in enumerate(PAIRS):
            for a, b in ((i, j), (j, i)):
                for c, d in ((k, l), (l, k)):
                    T[a, b, c, d] = C[I, J]
    return T


def sym_tensor(v):
    """(11,22,33,23,13,12) tensor components -> symmetric 3x3."""
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros((3, 3) + v.shape[1:], dtype=v.dtype)
    for I, (i, j) in enumerate(PAIRS):
        t[i, j] = v[I]
        t[j, i] = v[I]
    return t


def sym_vector(t):
    """symmetric 3x3 (leading axes) -> (11,22,33,23,13,12) components."""
    return np.stack([t[i, j] for (i, j) in PAIRS])


def frobenius(t):
    """Frobenius norm over all nine components of a 3x3 tensor."""
    return float(np.sqrt(np.sum(np.abs(t) ** 2)))


def solve_stiffness(C, Y):
    """X with C:X = Y for a Voigt stiffness C and a symmetric 3x3 tensor Y, i.e. the
    action of the inverse stiffness (compliance) on symmetric tensors.  Written in the
    Mandel basis, where the double contraction is an ordinary 6x6 product."""
    s = np.array([1, 1, 1, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])
    M = np.asarray(C, dtype=np.float64) * np.outer(s, s)
    y = sym_vector(np.asarray(Y, dtype=np.float64)) * s
    return sym_tensor(np.linalg.solve(M, y) / s)

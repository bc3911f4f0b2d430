"""Closed-form response of an axis-aligned laminate (test infrastructure only).

If the stiffness depends only on the coordinate along the unit axis n, the
discrete problem has the continuum laminate solution exactly: with u a
function of x_n only, both tetrahedral gradients of eqs. DA1-DA2 reduce to
the one-dimensional difference across a layer, so every layer p carries the
uniform strain Ebar + sym(a_p (x) n); the corner force (eq. L2-norm) is
2 (sigma_below - sigma_above).n, so equilibrium is traction continuity
sigma_p.n = t in all layers, and periodicity gives sum_p f_p a_p = 0.
With A_p,ik = C_p,ijkl n_j n_l and b_p = (C_p:Ebar).n:
    a_p = A_p^-1 (t - b_p),   t = (sum f_p A_p^-1)^-1 sum f_p A_p^-1 b_p.
"""
import numpy as np

from . import voigt


def mean_stress(C, fractions, axis, E):
    """<sigma> (tensor comps) of a laminate with normal along `axis` (0,1,2)."""
    n = np.zeros(3)
    n[axis] = 1.0
    Eb = voigt.sym_tensor(np.asarray(E, dtype=np.float64))
    Ct = [voigt.stiffness_tensor(c) for c in C]
    A = [np.einsum("ijkl,j,l->ik", c, n, n) for c in Ct]
    b = [np.einsum("ijkl,kl,j->i", c, Eb, n) for c in Ct]
    Ai = [np.linalg.inv(a) for a in A]
    S = sum(f * ai for f, ai in zip(fractions, Ai))
    t = np.linalg.solve(S, sum(f * ai @ bb for f, ai, bb in zip(fractions, Ai, b)))
    ms = np.zeros((3, 3))
    for f, c, ai, bb in zip(fractions, Ct, Ai, b):
        a = ai @ (t - bb)
        eps = Eb + 0.5 * (np.outer(a, n) + np.outer(n, a))
        ms += f * np.einsum("ijkl,kl->ij", c, eps)
    return voigt.sym_vector(ms)

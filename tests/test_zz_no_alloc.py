"""hz_solve_static: the solve on the library's static device workspace (no caller
workspace, no device allocation) gives what hz_solve gives on a bound workspace,
on two calls in a row, the second with a smaller input; and it refuses a problem
that does not fit the static array."""
import ctypes

import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz
from paper_2405_11168_amd import _abi

pytestmark = pytest.mark.gpu


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _problem(shape, seed):
    rng = np.random.default_rng(seed)
    N1, N2, N3 = shape
    ph = rng.integers(0, 3, (N3, N2, N1)).astype(np.uint16)
    C = np.stack([syn.random_spd_voigt(rng, 0.5, 8.0) for _ in range(3)])
    s = np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5])
    top = max(np.linalg.eigvalsh(c * np.outer(s, s)).max() for c in C)
    C0 = syn.isotropic_voigt(0.75 * top, 0.0)
    E = rng.normal(size=(2, 6)) * 1e-3
    return ph, C, C0, E


def _static_solve(g, E, o, fields):
    import torch

    nl = E.shape[0]
    n1, n2, n3 = g.shape
    sm = np.zeros((nl, 6))
    infos = (hz.hz_info * nl)()
    eps = np.zeros((nl, 6, n3, n2, n1)) if fields else None
    sig = np.zeros((nl, 6, n3, n2, n1)) if fields else None
    stream = torch.cuda.current_stream().cuda_stream
    rc = hz.lib().hz_solve_static(g._h, ctypes.c_void_p(stream), nl, _dp(E), ctypes.byref(o), _dp(sm),
                                  _dp(eps) if fields else None, _dp(sig) if fields else None, infos)
    _abi.check(rc)
    return rc, sm, infos, eps, sig


@pytest.mark.parametrize("precision", [hz.HZ_FP64, hz.HZ_FP32_REFINE], ids=["fp64", "fp32_refine"])
def test_static_workspace_solve_equals_bound_workspace_solve(precision):
    cases = [((32, 24, 20), 1, 2), ((16, 8, 12), 2, 1)]  # the second call is smaller
    for shape, seed, nl in cases:
        ph, C, C0, E = _problem(shape, seed)
        E = np.ascontiguousarray(E[:nl])
        g = hz.Grid(*shape)
        g.set_material(C, ph)
        fields = precision == hz.HZ_FP64
        ref = g.solve(E, tol=1e-9, C0=C0, precision=precision, fields=fields)
        o = hz._opts(tol=1e-9, precision=precision, C0=C0)
        rc, sm, infos, eps, sig = _static_solve(g, E, o, fields)
        iters = np.array([i.iters for i in infos])
        res = np.array([i.residual for i in infos])
        print(f"  static {shape} x{nl} precision {precision}: rc {rc} iters {iters} residual {res}", flush=True)
        assert rc == ref.rc
        assert np.array_equal(iters, ref.iters)
        assert np.array_equal(res, ref.residual)
        assert np.array_equal(sm, ref.mean_sigma)
        if fields:
            assert np.array_equal(eps, ref.eps) and np.array_equal(sig, ref.sigma)
        # the grid's own binding is untouched: its displacement is that of the bound solve
        u = g.displacement(0)
        again = g.solve(E, tol=1e-9, C0=C0, precision=precision)
        assert np.array_equal(again.mean_sigma, ref.mean_sigma)
        assert np.array_equal(g.displacement(0), u)


def test_static_workspace_refuses_a_problem_that_does_not_fit():
    g = hz.Grid(128, 128, 128)
    C = np.stack([syn.isotropic_voigt(1.0, 0.3)])
    g.set_material(C, np.zeros((128, 128, 128), dtype=np.uint16))
    assert g.workspace_bytes(hz.HZ_FP64, 1) > 256 << 20
    E = np.zeros((1, 6))
    E[0, 0] = 1e-3
    o = hz._opts()
    sm = np.zeros((1, 6))
    rc = hz.lib().hz_solve_static(g._h, None, 1, _dp(E), ctypes.byref(o), _dp(sm), None, None, None)
    assert rc == _abi.HZ_EWORKSPACE
    assert b"static workspace" in hz.lib().hz_last_error()

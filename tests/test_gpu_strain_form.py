"""GPU parity of the strain-based form (Algorithm 2: the 12 strain spectra are the
iterate, updated by Gamma(q).r) against the oracle's Algorithm 2 and Algorithm 1,
and against the GPU's own displacement-based forms, iterate by iterate.  Same
tolerances as the other FP64 parity tests."""
import numpy as np
import pytest

import paper_2405_11168_amd as hz
from oracle import tetra
from test_gpu_parity import random_problem

pytestmark = pytest.mark.gpu

STRAIN = hz.HZ_SCHEME_STRAIN


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("shape,n_phases,seed,kind,voids,K", [
    ((16, 16, 16), 2, 50, "iso", False, 6),
    ((12, 10, 8), 3, 51, "aniso", False, 5),
    ((12, 6, 20), 3, 52, "aniso", True, 5),
    ((40, 30, 18), 2, 53, "iso", False, 3),
])
def test_strain_form_iterates_match_oracle(shape, n_phases, seed, kind, voids, K):
    ph, C, C0, E = random_problem(shape, n_phases, seed, kind, voids)
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    r = g.solve(E, C0=C0, fixed_iters=K, trace=True, fields=True, scheme=STRAIN)
    h2, m2 = tetra.strain_scheme(ph, C, C0, E[0], K)
    ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=K)
    eh = np.max(np.abs(r.trace_residual[0, : K + 1] - h2) / h2)
    em = np.abs(r.trace_mean[0, : K + 1] - m2).max() / np.abs(m2).max()
    es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
    ee = np.abs(r.eps[0] - ref.eps).max() / np.abs(ref.eps).max()
    _say(f"  strain form {shape} K={K}: residual {eh:.2e} <sigma> {em:.2e} sigma {es:.2e} eps {ee:.2e}")
    assert r.status[0] == hz.HZ_OK and r.iters[0] == K
    assert eh < 1e-10 and em < 1e-12 and es < 1e-11 and ee < 1e-11


def test_strain_form_equals_displacement_forms_to_tol():
    """Run to tol: the same stop iterate and <sigma> to rounding as the Fourier and
    stencil forms, for six loads at once (C_eff)."""
    ph, C, C0, _ = random_problem((16, 12, 10), 3, 54, "aniso")
    g = hz.Grid(16, 12, 10)
    g.set_material(C, ph)
    Cs, rs = g.effective_stiffness(tol=1e-10, C0=C0, scheme=STRAIN)
    for scheme in (hz.HZ_SCHEME_SPECTRAL, hz.HZ_SCHEME_STENCIL):
        Cd, rd = g.effective_stiffness(tol=1e-10, C0=C0, scheme=scheme)
        err = np.abs(Cs - Cd).max() / np.abs(Cd).max()
        _say(f"  scheme {scheme}: iters {rd.iters} vs strain form {rs.iters}, C_eff diff {err:.2e}")
        assert np.array_equal(rs.iters, rd.iters)
        assert err < 1e-12


def test_strain_form_with_applied_stress_and_eigenstrain():
    shape = (12, 10, 16)
    ph, C, C0, _ = random_problem(shape, 3, 55, "aniso")
    rng = np.random.default_rng(55)
    e0 = rng.normal(size=(3, 6)) * 5e-3
    e0[0] = 0.0
    sa = np.array([[0.4, -0.1, 0.2, 0.05, -0.08, 0.12]])
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    g.set_eigenstrain(e0)
    K = 6
    r = g.solve(sa, C0=C0, fixed_iters=K, trace=True, fields=True, scheme=STRAIN, loading=hz.HZ_LOAD_STRESS)
    ref = tetra.basic_scheme(ph, C, C0, sa[0], fixed_iters=K, eps0=e0, stress=True)
    eh = np.max(np.abs(r.trace_residual[0, : K + 1] - ref.history) / ref.history)
    em = np.abs(r.trace_mean[0, : K + 1] - ref.mean_history).max() / np.abs(ref.mean_history).max()
    eb = np.abs(r.Ebar[0] - ref.Ebar).max() / np.abs(ref.Ebar).max()
    es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
    _say(f"  strain form, stress + eigenstrain: residual {eh:.2e} <sigma> {em:.2e} Ebar {eb:.2e} sigma {es:.2e}")
    assert eh < 1e-10 and em < 1e-12 and eb < 1e-12 and es < 1e-11


def test_strain_form_api_limits():
    ph, C, C0, E = random_problem((8, 8, 8), 2, 56, "iso")
    g = hz.Grid(8, 8, 8)
    g.set_material(C, ph)
    g.solve(E, C0=C0, tol=1e-8, scheme=STRAIN)
    with pytest.raises(hz.HzError) as e:
        g.displacement(0)
    assert e.value.code == hz._abi.HZ_EINVAL
    with pytest.raises(hz.HzError) as e:
        g.solve(E, C0=C0, tol=1e-8, scheme=STRAIN, precision=hz.HZ_FP32_REFINE)
    assert e.value.code == hz._abi.HZ_EINVAL
    srv = hz.Server(hz.request_bytes(g, hz.HZ_FP64, 1), max_problems=2)
    with pytest.raises(hz.HzError) as e:
        srv.submit(g, E, C0=C0, scheme=STRAIN)
    assert e.value.code == hz._abi.HZ_EINVAL

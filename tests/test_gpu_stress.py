"""GPU parity of the applied-stress loop (Sec. 2.5, step 6 of Algorithm 1) and of
eigenstrains, through the C ABI, against the FP64 oracle on the same seeded inputs.

Tolerances as for strain loading: eps_k to 1e-10 relative, <sigma>_k and the mean
strain to 1e-12 of their scale, u and the fields to 1e-11.  The device applies step
6 in the equivalent form Ebar += lambda0^-1:(sigma^a - <sigma>_k); the oracle
evaluates the printed formula, so the two differ by rounding only."""
import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz
from oracle import tetra
from test_gpu_parity import SCHEMES, oracle_u_in_library_layout, random_problem

pytestmark = pytest.mark.gpu

S_A = np.array([[0.4, -0.1, 0.2, 0.05, -0.08, 0.12]])


def _say(msg):
    print(msg, flush=True)


def _eig(n_phases, seed):
    rng = np.random.default_rng(seed)
    e0 = rng.normal(size=(n_phases, 6)) * 5e-3
    e0[0] = 0.0
    return e0


def _grid(shape, C, ph, eps0=None):
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    if eps0 is not None:
        g.set_eigenstrain(eps0)
    return g


def _check(shape, g, r, ref, K, fields):
    assert r.status[0] == hz.HZ_OK and r.iters[0] == K
    eh = np.max(np.abs(r.trace_residual[0, : K + 1] - ref.history) / ref.history)
    scale = np.abs(ref.mean_history).max()
    em = np.abs(r.trace_mean[0, : K + 1] - ref.mean_history).max() / scale
    eb = np.abs(r.Ebar[0] - ref.Ebar).max() / np.abs(ref.Ebar).max()
    u = g.displacement(0)
    uo = oracle_u_in_library_layout(ref.u_hat, shape)
    eu = np.abs(u - uo).max() / max(np.abs(uo).max(), 1e-300)
    _say(f"  shape {shape} K={K}: residual hist {eh:.2e}  <sigma> {em:.2e}  Ebar {eb:.2e}  u {eu:.2e}")
    assert eh < 1e-10 and em < 1e-12 and eb < 1e-12 and eu < 1e-11
    if fields:
        es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
        ee = np.abs(r.eps[0] - ref.eps).max() / np.abs(ref.eps).max()
        _say(f"  fields: sigma {es:.2e} eps {ee:.2e}")
        assert es < 1e-11 and ee < 1e-11


@pytest.mark.parametrize("shape,n_phases,seed,kind,voids,eig,K", [
    ((12, 10, 16), 3, 31, "aniso", False, True, 6),
    ((16, 16, 16), 2, 32, "iso", False, True, 6),    # isotropic kernels with eigenstress
    ((32, 48, 40), 2, 33, "iso", False, False, 4),   # several tiles, stress only
    ((12, 6, 20), 3, 34, "aniso", True, True, 5),    # voids
])
@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_stress_loading_iterates_match_oracle(shape, n_phases, seed, kind, voids, eig, K, scheme):
    _say(f"case stress shape={shape} seed={seed} kind={kind} voids={voids} eig={eig} scheme={scheme}")
    ph, C, C0, _ = random_problem(shape, n_phases, seed, kind, voids)
    e0 = _eig(n_phases, seed) if eig else None
    g = _grid(shape, C, ph, e0)
    if not g.scheme_available(scheme):
        pytest.skip(f"scheme {scheme} not available for {shape}")
    r = g.solve(S_A, C0=C0, fixed_iters=K, trace=True, fields=True, scheme=scheme, loading=hz.HZ_LOAD_STRESS)
    ref = tetra.basic_scheme(ph, C, C0, S_A[0], fixed_iters=K, eps0=e0, stress=True)
    _check(shape, g, r, ref, K, True)


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_strain_loading_with_eigenstrain_matches_oracle(scheme):
    shape = (20, 12, 14)
    ph, C, C0, E = random_problem(shape, 3, 35, "aniso")
    e0 = _eig(3, 35)
    g = _grid(shape, C, ph, e0)
    if not g.scheme_available(scheme):
        pytest.skip(f"scheme {scheme} not available for {shape}")
    r = g.solve(E, C0=C0, fixed_iters=5, trace=True, fields=True, scheme=scheme)
    ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=5, eps0=e0)
    _check(shape, g, r, ref, 5, True)
    assert np.array_equal(r.Ebar[0], E[0])


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_stress_loading_converges_to_the_oracle_solution(scheme):
    """Run to tol: the same stop iterate as the oracle, <sigma> = sigma^a, and the mean
    strain of that iterate."""
    shape = (16, 12, 10)
    ph, C, C0, _ = random_problem(shape, 3, 36, "aniso")
    e0 = _eig(3, 36)
    g = _grid(shape, C, ph, e0)
    if not g.scheme_available(scheme):
        pytest.skip(f"scheme {scheme} not available for {shape}")
    r = g.solve(S_A, C0=C0, tol=1e-9, scheme=scheme, loading=hz.HZ_LOAD_STRESS)
    ref = tetra.basic_scheme(ph, C, C0, S_A[0], tol=1e-9, eps0=e0, stress=True, keep_fields=False)
    _say(f"  iters gpu {r.iters[0]} oracle {ref.iters}, res {r.residual[0]:.3e}")
    assert r.status[0] == hz.HZ_OK and ref.converged
    assert abs(int(r.iters[0]) - ref.iters) <= 1
    assert np.abs(r.mean_sigma[0] - S_A[0]).max() <= 1e-8 * np.abs(S_A).max()
    refk = tetra.basic_scheme(ph, C, C0, S_A[0], fixed_iters=int(r.iters[0]), eps0=e0, stress=True,
                              keep_fields=False)
    assert np.abs(r.Ebar[0] - refk.Ebar).max() < 1e-12 * np.abs(refk.Ebar).max()


def test_eigenstrain_inclusion_under_zero_applied_stress():
    """A cubic inclusion with an eigenstrain eps0_33 in a homogeneous isotropic cell
    under zero applied stress (the set-up of Sec. 3.3): the mean strain is the mean
    eigenstrain exactly and <sigma> vanishes."""
    shape = (24, 24, 24)
    ph = np.zeros((24, 24, 24), dtype=np.uint16)
    ph[8:16, 8:16, 8:16] = 1
    Cm = syn.isotropic_voigt(1.0, 0.3)
    C = np.stack([Cm, Cm])
    e0 = np.zeros((2, 6))
    e0[1, 2] = 0.01
    C0 = syn.isotropic_voigt(1.65, 0.0)  # Mandel modulus midway between 2 mu and 3 K of the cell
    g = _grid(shape, C, ph, e0)
    r = g.solve(np.zeros((1, 6)), C0=C0, tol=1e-10, loading=hz.HZ_LOAD_STRESS, fields=True)
    f = np.mean(ph == 1)
    _say(f"  iters {r.iters[0]} Ebar {r.Ebar[0]} <sigma> {r.mean_sigma[0]}")
    assert r.status[0] == hz.HZ_OK
    assert np.abs(r.Ebar[0] - f * e0[1]).max() < 1e-12
    assert np.abs(r.mean_sigma[0]).max() < 1e-12
    ref = tetra.basic_scheme(ph, C, C0, np.zeros(6), fixed_iters=int(r.iters[0]), eps0=e0, stress=True)
    es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
    _say(f"  sigma field vs oracle at the same iterate {es:.2e}")
    assert es < 1e-11


def test_fp32_refine_with_eigenstrain():
    p = syn.sphere16()
    e0 = np.zeros((2, 6))
    e0[1] = [0.002, 0.002, 0.002, 0.0, 0.0, 0.0]
    g = _grid(p.shape, p.C, p.phase, e0)
    E = np.stack([p.loads[0], 1e-3 * syn.unit_load(4)])
    r = g.solve(E, C0=p.C0, tol=1e-8, precision=hz.HZ_FP32_REFINE)
    _say(f"  refine+eig: status {r.status} iters {r.iters} rounds {r.outer_rounds} res {r.residual}")
    assert np.all(r.status == hz.HZ_OK) and np.all(r.residual < 1e-8)
    for J in range(2):
        ref = tetra.basic_scheme(p.phase, p.C, p.C0, E[J], tol=1e-12, eps0=e0, keep_fields=False)
        err = np.abs(r.mean_sigma[J] - ref.mean_sigma).max() / np.abs(ref.mean_sigma).max()
        _say(f"  load {J}: <sigma> rel err {err:.2e}")
        assert err < 1e-6


def test_server_mixes_stress_eigenstrain_and_strain_requests_bitwise():
    """Problems of all four material kinds (isotropic or not, with or without
    eigenstrains) and both loadings in one serving group give what each gives alone."""
    shape = (16, 16, 16)
    grids, reqs = [], []
    for i, (kind, eig, loading) in enumerate([("iso", False, hz.HZ_LOAD_STRAIN), ("iso", True, hz.HZ_LOAD_STRESS),
                                              ("aniso", False, hz.HZ_LOAD_STRESS), ("aniso", True, hz.HZ_LOAD_STRAIN)]):
        ph, C, C0, E = random_problem(shape, 2, 40 + i, kind)
        g = _grid(shape, C, ph, _eig(2, 40 + i) if eig else None)
        grids.append(g)
        load = S_A if loading == hz.HZ_LOAD_STRESS else E
        reqs.append((g, load, C0, loading))
    alone = []
    for g, load, C0, loading in reqs:
        srv = hz.Server(hz.request_bytes(g, hz.HZ_FP64, 1), max_problems=4)
        rid = srv.submit(g, load, C0=C0, tol=1e-9, loading=loading)
        srv.drain()
        alone.append(srv.result(rid))
    total = sum(hz.request_bytes(g, hz.HZ_FP64, 1) for g, *_ in reqs)
    srv = hz.Server(int(1.2 * total), max_problems=8, check_every=4)
    ids = [srv.submit(g, load, C0=C0, tol=1e-9, loading=loading) for g, load, C0, loading in reqs]
    srv.drain()
    for i, rid in enumerate(ids):
        r = srv.result(rid)
        _say(f"  request {i}: iters {r.iters} res {r.residual} Ebar {r.Ebar[0][:3]}")
        assert r.rc == hz.HZ_OK
        assert np.array_equal(r.mean_sigma, alone[i].mean_sigma) and np.array_equal(r.iters, alone[i].iters)
        assert np.array_equal(r.Ebar, alone[i].Ebar) and np.array_equal(r.residual, alone[i].residual)
        g, load, C0, loading = reqs[i]
        rs = g.solve(load, C0=C0, tol=1e-9, loading=loading)
        assert np.array_equal(rs.mean_sigma, r.mean_sigma) and np.array_equal(rs.Ebar, r.Ebar)


def test_full_size_boolean128_under_applied_stress_first_iterates():
    """The 128^3 Boolean workload of the benchmark under an applied stress (stencil
    form, six loads at once): iterates 0..2 of one load against the oracle."""
    p = syn.boolean128()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    loads = np.zeros((6, 6))
    loads[:, :] = S_A[0]
    loads[1:] *= np.arange(2, 7)[:, None]  # six different stress levels
    K = 2
    r = g.solve(loads, C0=p.C0, fixed_iters=K, trace=True, loading=hz.HZ_LOAD_STRESS)
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, loads[3], fixed_iters=K, stress=True, keep_fields=False)
    eh = np.max(np.abs(r.trace_residual[3, : K + 1] - ref.history) / ref.history)
    em = np.abs(r.trace_mean[3, : K + 1] - ref.mean_history).max() / np.abs(ref.mean_history).max()
    eb = np.abs(r.Ebar[3] - ref.Ebar).max() / np.abs(ref.Ebar).max()
    _say(f"  boolean128 stress: residual {eh:.2e} <sigma> {em:.2e} Ebar {eb:.2e}")
    assert eh < 1e-10 and em < 1e-12 and eb < 1e-12

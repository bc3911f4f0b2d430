"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, iterate by iterate.

Tolerances (FP64 path): the residual history eps_k to 1e-10 relative and
<sigma>_k to 1e-12 of its scale, the displacement spectrum and the final
fields to 1e-11 of their scale.  Both sides run Algorithm 1 in FP64 with
different FFT factorisations and summation orders, so they agree to a small
multiple of machine epsilon times the contrast.
"""
import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz
from oracle import tetra

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def phase_factor(shape):
    """exp(i q.(1/2,1/2,1/2)) on the half spectrum [h1, h3, h2] (library convention)."""
    N1, N2, N3 = shape
    h1 = np.arange(N1 // 2 + 1)[:, None, None]
    h3 = np.arange(N3)[None, :, None]
    h2 = np.arange(N2)[None, None, :]
    return np.exp(1j * np.pi * (h1 / N1 + h2 / N2 + h3 / N3))


def oracle_u_in_library_layout(u_hat, shape):
    """oracle u(q) [3, N3, N2, N1] -> [3, N1/2+1, N3, N2] times the corner phase."""
    N1 = shape[0]
    half = u_hat[:, :, :, : N1 // 2 + 1]  # [3, h3, h2, h1]
    return np.transpose(half, (0, 3, 1, 2)) * phase_factor(shape)[None]


def random_problem(shape, n_phases, seed, kind="aniso", voids=False):
    rng = np.random.default_rng(seed)
    N1, N2, N3 = shape
    ph = rng.integers(0, n_phases, (N3, N2, N1)).astype(np.uint16)
    if kind == "aniso":
        C = np.stack([syn.random_spd_voigt(rng, 0.5, 8.0) for _ in range(n_phases)])
    else:
        C = np.stack([syn.isotropic_voigt(float(E), 0.3) for E in 10.0 ** rng.uniform(0, 2, n_phases)])
    if voids:
        C[-1] = 0.0
    s = np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5])
    top = max(np.linalg.eigvalsh(c * np.outer(s, s)).max() for c in C)
    C0 = syn.isotropic_voigt(0.75 * top, 0.0)
    E = np.array([[1e-3, -2e-4, 3e-4, 1e-4, -5e-4, 2e-4]])
    return ph, C, C0, E


SCHEMES = [hz.HZ_SCHEME_SPECTRAL, hz.HZ_SCHEME_STENCIL]


def run_pair(shape, ph, C, C0, E, K, fields=True, scheme=hz.HZ_SCHEME_SPECTRAL):
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    if not g.scheme_available(scheme):
        pytest.skip(f"scheme {scheme} not available for {shape}")
    r = g.solve(E, precision=hz.HZ_FP64, C0=C0, fixed_iters=K, trace=True, fields=fields, scheme=scheme)
    ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=K, keep_fields=fields)
    return g, r, ref


def check_pair(shape, g, r, ref, K, fields=True):
    assert r.status[0] == hz.HZ_OK and r.iters[0] == K
    eh = np.max(np.abs(r.trace_residual[0, : K + 1] - ref.history) / ref.history)
    scale = np.abs(ref.mean_history).max()
    em = np.abs(r.trace_mean[0, : K + 1] - ref.mean_history).max() / scale
    u = g.displacement(0)
    uo = oracle_u_in_library_layout(ref.u_hat, shape)
    eu = np.abs(u - uo).max() / max(np.abs(uo).max(), 1e-300)
    _say(f"  shape {shape} K={K}: residual hist {eh:.2e}  <sigma> {em:.2e}  u {eu:.2e}")
    assert eh < 1e-10
    assert em < 1e-12
    assert eu < 1e-11
    if fields:
        es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
        ee = np.abs(r.eps[0] - ref.eps).max() / np.abs(ref.eps).max()
        _say(f"  fields: sigma {es:.2e} eps {ee:.2e}")
        assert es < 1e-11 and ee < 1e-11


@pytest.mark.parametrize("shape,n_phases,seed,kind,voids,K", [
    ((16, 16, 16), 2, 0, "iso", False, 8),
    ((6, 10, 12), 3, 1, "aniso", False, 6),      # radix 3 (N1/2), 5, 3
    ((12, 6, 20), 3, 2, "aniso", True, 6),       # voids
    ((14, 8, 28), 2, 3, "iso", False, 4),        # radix 7
    ((2, 4, 6), 2, 4, "aniso", False, 5),        # degenerate N1 = 2
    ((32, 48, 40), 2, 5, "iso", False, 4),       # several tiles in every pass, ragged y tile
    ((40, 30, 18), 3, 6, "aniso", False, 3),
    ((128, 16, 16), 2, 7, "iso", False, 3),      # x tile larger than one load batch; radix 16 x 4
    ((64, 32, 32), 2, 8, "aniso", False, 3),     # radix 16 x 2 along x
    ((256, 8, 8), 2, 9, "iso", False, 2),        # radix 16 x 8 along x, narrow y/z
    ((16, 256, 8), 2, 10, "iso", False, 2),      # radix 16 x 16 along y
    ((16, 8, 256), 2, 11, "iso", False, 2),      # radix 16 x 16 along z
    ((96, 48, 40), 2, 12, "aniso", True, 3),     # radix 3 and 5 at medium size, voids
    # N1 a multiple of 64 with few rows and planes: ragged stencil tiles along y, z segments
    # shorter than a tile, three-pass x transforms
    ((64, 12, 10), 2, 13, "iso", False, 3),
    ((128, 20, 6), 3, 14, "aniso", True, 3),
    ((192, 14, 4), 2, 15, "iso", True, 2),
    ((64, 4, 2), 2, 16, "aniso", False, 3),
    ((320, 6, 4), 2, 17, "iso", False, 2),
    # N1/2 without a factor 2: the stencil form's x transforms split and merge on an odd
    # radix (15 = 3 then 5, 9 = 3 x 3, 63 = 3, 7, 3) or in one pass (5)
    ((30, 12, 10), 3, 18, "aniso", False, 4),
    ((18, 20, 6), 2, 19, "aniso", True, 4),
    ((126, 8, 6), 2, 20, "iso", False, 3),
    ((10, 6, 8), 2, 21, "iso", True, 5),
    ((126, 96, 80), 3, 22, "aniso", False, 2),   # odd split radix over many tiles (63 = 3, 7, 3)
    # z tiles whose LDS exceeds 64 KB: 4 FP64 columns of N3 = 320 (66.5 KB), and the longest
    # z lines, N3 = 1080 (one column, 67.5 KB)
    ((8, 8, 320), 2, 24, "aniso", False, 2),
    ((6, 4, 1080), 2, 25, "iso", True, 2),
    ((8, 2016, 8), 2, 23, "iso", False, 2),      # longest y lines: FP64 lines unpadded in LDS
])
@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_fp64_iterates_match_oracle(shape, n_phases, seed, kind, voids, K, scheme):
    _say(f"case shape={shape} seed={seed} kind={kind} voids={voids} scheme={scheme}")
    ph, C, C0, E = random_problem(shape, n_phases, seed, kind, voids)
    g, r, ref = run_pair(shape, ph, C, C0, E, K, scheme=scheme)
    check_pair(shape, g, r, ref, K)


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_fully_anisotropic_reference_medium(scheme):
    """Generic (non-isotropic) reference medium: the Green operator path that contracts
    the full lambda0 tensor (eq. Green_tensor) rather than the isotropic closed form."""
    shape = (12, 10, 16)
    ph, C, _, E = random_problem(shape, 3, 21, "aniso")
    rng = np.random.default_rng(22)
    C0 = syn.random_spd_voigt(rng, 6.0, 14.0)
    g, r, ref = run_pair(shape, ph, C, C0, E, 4, scheme=scheme)
    check_pair(shape, g, r, ref, 4)


def test_sphere16_converged_ceff_matches_oracle_iterate_matched():
    """16^3 centred sphere, contrast 10: GPU C_eff at its stop iterate vs the oracle at
    the same iterate (<= 1e-10 relative), and the same stop iterate up to one step."""
    p = syn.sphere16()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    Ce, r = g.effective_stiffness(tol=p.tol, C0=p.C0, trace=True)
    assert np.all(r.status == hz.HZ_OK)
    cols = []
    for J in range(6):
        E = syn.unit_load(J)
        ref = tetra.basic_scheme(p.phase, p.C, p.C0, E, tol=p.tol, keep_fields=False)
        assert abs(ref.iters - r.iters[J]) <= 1
        refk = tetra.basic_scheme(p.phase, p.C, p.C0, E, fixed_iters=int(r.iters[J]), keep_fields=False)
        cols.append(refk.mean_sigma)
    Co = np.array(cols).T
    err = np.abs(Ce - Co).max() / np.abs(Co).max()
    _say(f"  sphere16 C_eff rel err {err:.2e}, iters {r.iters}")
    assert err < 1e-10


def test_effective_stiffness_entry_equals_six_unit_solves_bitwise():
    """hz_effective_stiffness (the C-ABI call Grid.effective_stiffness makes) returns as
    column J exactly <sigma> of hz_solve on the unit load gamma_J = 1."""
    ph, C, C0, _ = random_problem((16, 12, 10), 3, 31, "aniso")
    g = hz.Grid(16, 12, 10)
    g.set_material(C, ph)
    for prec in (hz.HZ_FP64, hz.HZ_FP32_REFINE):
        Ce, r = g.effective_stiffness(tol=1e-9, C0=C0, precision=prec)
        E = np.array([syn.unit_load(J) for J in range(6)])
        rs = g.solve(E, tol=1e-9, C0=C0, precision=prec)
        assert np.array_equal(Ce, rs.mean_sigma.T), prec
        assert np.array_equal(r.iters, rs.iters) and np.array_equal(r.residual, rs.residual)
        asym = np.abs(Ce - Ce.T).max() / np.abs(Ce).max()
        _say(f"  C_eff precision {prec}: iters {r.iters}, symmetry residual {asym:.1e}")
        assert asym < 1e-7


def test_device_field_outputs_equal_host_outputs():
    """fields_on_device: eps and sigma written into caller-owned device arrays equal the
    host outputs bit for bit, for a batch of loads in both forms."""
    ph, C, C0, E = random_problem((16, 12, 10), 2, 32, "aniso")
    E = np.vstack([E, 0.5 * E[:, ::-1]])
    g = hz.Grid(16, 12, 10)
    g.set_material(C, ph)
    for scheme in SCHEMES:
        rh = g.solve(E, C0=C0, fixed_iters=5, fields=True, scheme=scheme)
        rd = g.solve(E, C0=C0, fixed_iters=5, fields=True, fields_on_device=True, scheme=scheme)
        assert rd.eps.is_cuda and rd.eps.shape == rh.eps.shape
        assert np.array_equal(rd.eps.cpu().numpy(), rh.eps) and np.array_equal(rd.sigma.cpu().numpy(), rh.sigma)


def test_batched_loads_equal_single_loads_bitwise():
    ph, C, C0, _ = random_problem((12, 10, 8), 3, 7, "aniso")
    E = np.array([syn.unit_load(J) for J in range(6)]) * 1e-3
    g = hz.Grid(12, 10, 8)
    g.set_material(C, ph)
    rb = g.solve(E, C0=C0, tol=1e-9, trace=True)
    for J in (0, 4):
        rs = g.solve(E[J:J + 1], C0=C0, tol=1e-9, trace=True)
        assert rs.iters[0] == rb.iters[J]
        assert np.array_equal(rs.mean_sigma[0], rb.mean_sigma[J])


def _u_err(g, J, ref, shape):
    """max |u_gpu - u_oracle| / max |u_oracle| over the whole half spectrum of load J."""
    uo = oracle_u_in_library_layout(ref.u_hat, shape)
    return np.abs(g.displacement(J) - uo).max() / np.abs(uo).max()


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_full_size_boolean128_first_iterates(scheme):
    """The 128^3 Boolean-sphere workload (contrast 1e3, 6 loads) in the launch
    configuration the benchmark times: iterates 0..2 of two loads vs the oracle,
    residual and <sigma> at every iterate and the displacement u_2 element by element."""
    p = syn.boolean128()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    K = 2
    r = g.solve(p.loads, precision=hz.HZ_FP64, C0=p.C0, fixed_iters=K, trace=True, scheme=scheme)
    for J in (0, 5):
        ref = tetra.basic_scheme(p.phase, p.C, p.C0, p.loads[J], fixed_iters=K, keep_fields=False)
        eh = np.max(np.abs(r.trace_residual[J, : K + 1] - ref.history) / ref.history)
        em = np.abs(r.trace_mean[J, : K + 1] - ref.mean_history).max() / np.abs(ref.mean_history).max()
        eu = _u_err(g, J, ref, p.shape)
        _say(f"  boolean128 load {J}: residual hist {eh:.2e} <sigma> {em:.2e} u {eu:.2e}")
        assert eh < 1e-10 and em < 1e-12 and eu < 1e-11


def test_full_size_boolean128_fields_one_load():
    """The 128^3 workload: the fields of eq. final_fields of one load after 2 updates,
    every voxel and component against the oracle (host and device outputs)."""
    p = syn.boolean128()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    K = 2
    E = p.loads[:1]
    r = g.solve(E, C0=p.C0, fixed_iters=K, fields=True)
    rd = g.solve(E, C0=p.C0, fixed_iters=K, fields=True, fields_on_device=True)
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, E[0], fixed_iters=K, keep_fields=True)
    es = np.abs(r.sigma[0] - ref.sigma).max() / np.abs(ref.sigma).max()
    ee = np.abs(r.eps[0] - ref.eps).max() / np.abs(ref.eps).max()
    _say(f"  boolean128 fields: sigma {es:.2e} eps {ee:.2e}")
    assert es < 1e-11 and ee < 1e-11
    assert np.array_equal(rd.eps.cpu().numpy(), r.eps) and np.array_equal(rd.sigma.cpu().numpy(), r.sigma)


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_fp32_refine_ceff_within_1e6_of_converged_oracle(scheme):
    p = syn.sphere16()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    Ce, r = g.effective_stiffness(tol=1e-8, C0=p.C0, precision=hz.HZ_FP32_REFINE, scheme=scheme)
    _say(f"  refine: status {r.status} inner iters {r.iters} rounds {r.outer_rounds} res {r.residual}")
    assert np.all(r.status == hz.HZ_OK)
    assert np.all(r.residual < 1e-8)
    Co, _ = tetra.effective_stiffness(p.phase, p.C, p.C0, tol=1e-12)
    err = np.abs(Ce - Co).max() / np.abs(Co).max()
    _say(f"  refine C_eff rel err {err:.2e}")
    assert err < 1e-6


def test_fp32_refine_stencil_form_matches_converged_oracle():
    """FP32+refine in the stencil form on a grid with several stencil tiles per row and
    plane (FP32 iterations and FP64 sweeps): <sigma> within 1e-6 of the converged oracle,
    for an isotropic and an anisotropic material."""
    for seed, kind in ((41, "iso"), (42, "aniso")):
        ph, C, C0, E = random_problem((64, 16, 12), 2, seed, kind)
        g = hz.Grid(64, 16, 12)
        g.set_material(C, ph)
        r = g.solve(E, tol=1e-9, C0=C0, precision=hz.HZ_FP32_REFINE, scheme=hz.HZ_SCHEME_STENCIL)
        ref = tetra.basic_scheme(ph, C, C0, E[0], tol=1e-12, keep_fields=False)
        err = np.abs(r.mean_sigma[0] - ref.mean_sigma).max() / np.abs(ref.mean_sigma).max()
        _say(f"  refine stencil form {kind}: status {r.status[0]} iters {r.iters[0]} rounds {r.outer_rounds[0]} "
             f"<sigma> vs converged {err:.1e}")
        assert r.status[0] == hz.HZ_OK and err < 1e-6


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_fp32_fixed_count_matches_oracle_iterate(scheme):
    """A fixed FP32 count (fixed_iters = K with HZ_FP32_REFINE): K FP32 updates from u = 0,
    then one FP64 sweep measures the iterate.  Its <sigma> and eps against the oracle's
    iterate K, to the 1e-6 relative bound stated for FP32 fields: every FP32 pass rounds
    the fields by a few units of 2^-24 (6e-8), and the scheme is a contraction, so the
    FP32 iterate stays within a small multiple of that of the FP64 one."""
    for shape, seed, kind, K in (((64, 16, 12), 51, "iso", 12), ((32, 48, 40), 52, "aniso", 10),
                                 ((30, 12, 10), 53, "aniso", 8), ((14, 8, 28), 54, "iso", 8)):
        ph, C, C0, E = random_problem(shape, 3, seed, kind)
        g = hz.Grid(*shape)
        g.set_material(C, ph)
        if not g.scheme_available(scheme):
            continue
        r = g.solve(E, C0=C0, precision=hz.HZ_FP32_REFINE, fixed_iters=K, scheme=scheme)
        ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=K, keep_fields=False)
        em = np.abs(r.mean_sigma[0] - ref.mean_sigma).max() / np.abs(ref.mean_sigma).max()
        eh = abs(r.residual[0] - ref.history[K]) / ref.history[0]
        _say(f"  FP32 fixed count {shape} {kind} K={K}: <sigma> {em:.1e}, eps {eh:.1e} "
             f"(eps_K {ref.history[K]:.2e})")
        assert r.status[0] == hz.HZ_OK and r.iters[0] == K and r.outer_rounds[0] == 1
        assert em < 1e-6 and eh < 1e-6
    with pytest.raises(hz.HzError):
        g.solve(E, C0=C0, precision=hz.HZ_FP32_REFINE, fixed_iters=0, scheme=scheme)


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_fp32_refine_displacement_matches_converged_oracle(scheme):
    """The displacement an FP32+refine solve reports is its FP64 anchor U as u(q) (the
    stencil form holds U as its inverse z transform while it iterates)."""
    p = syn.sphere16()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    r = g.solve(p.loads[:1], tol=1e-9, C0=p.C0, precision=hz.HZ_FP32_REFINE, scheme=scheme)
    assert r.status[0] == hz.HZ_OK
    u = g.displacement(0)
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, p.loads[0], tol=1e-12, keep_fields=False)
    uo = oracle_u_in_library_layout(ref.u_hat, p.shape)
    eu = np.abs(u - uo).max() / np.abs(uo).max()
    _say(f"  refine displacement rel err {eu:.2e} (residual {r.residual[0]:.2e})")
    assert eu < 1e-6


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_large_non_power_of_two_cell_first_iterates(scheme):
    """The 192 x 192 x 320 cell (11.8 M voxels, radix 3 and 5 passes, narrow z tiles),
    Boolean spheres to 25% with contrast 1e2: iterates 0..1 against the oracle."""
    p = syn.sphere_contrast((192, 192, 320), 1e2)
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    if not g.scheme_available(scheme):
        pytest.skip(f"scheme {scheme} not available")
    K = 1
    E = p.loads[:1]
    r = g.solve(E, C0=p.C0, fixed_iters=K, trace=True, scheme=scheme)
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, E[0], fixed_iters=K, keep_fields=False)
    eh = np.max(np.abs(r.trace_residual[0, : K + 1] - ref.history) / ref.history)
    em = np.abs(r.trace_mean[0, : K + 1] - ref.mean_history).max() / np.abs(ref.mean_history).max()
    eu = _u_err(g, 0, ref, p.shape)
    _say(f"  192x192x320: residual hist {eh:.2e} <sigma> {em:.2e} u {eu:.2e}")
    assert eh < 1e-10 and em < 1e-12 and eu < 1e-11


def _full_size_iterates_both_forms(p, E, K, label):
    """Iterates 0..K of one load in both forms against one oracle run."""
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    _say(f"  {label}: oracle, {K} iteration(s) of {np.prod(p.shape)} voxels")
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, E[0], fixed_iters=K, keep_fields=False)
    for scheme in SCHEMES:
        if not g.scheme_available(scheme):
            continue
        r = g.solve(E, C0=p.C0, fixed_iters=K, trace=True, scheme=scheme)
        eh = np.max(np.abs(r.trace_residual[0, : K + 1] - ref.history) / ref.history)
        em = np.abs(r.trace_mean[0, : K + 1] - ref.mean_history).max() / np.abs(ref.mean_history).max()
        eu = _u_err(g, 0, ref, p.shape)
        _say(f"  {label} scheme {scheme}: residual hist {eh:.2e} <sigma> {em:.2e} u {eu:.2e}")
        assert eh < 1e-10 and em < 1e-12 and eu < 1e-11


def test_voronoi256_polycrystal_first_iterates():
    """The 256^3 Voronoi polycrystal (200 rotated cubic grains: every phase anisotropic,
    the time-to-1e-6 benchmark cell), a shear load: iterates 0..1 against the oracle."""
    p = syn.polycrystal()
    _full_size_iterates_both_forms(p, p.loads[3:4], 1, "voronoi256")


def test_stiff_endpoint_first_iterates():
    """The 192 x 192 x 320 sphere cell at contrast 1e8, the stiff end of the contrast sweep
    (the 256^3 voids test below is the soft end): iterates 0..1 against the oracle."""
    p = syn.sphere_contrast((192, 192, 320), 1e8)
    _full_size_iterates_both_forms(p, p.loads[:1], 1, "192x192x320 C=1e8")


def test_spheres256_voids_first_iterates():
    """256^3 Boolean spheres to 25% as voids (zero stiffness), the infinite-contrast cell:
    iterates 0..1 against the oracle."""
    p = syn.sphere_contrast((256, 256, 256), 0.0)
    _full_size_iterates_both_forms(p, p.loads, 1, "spheres256 voids")

"""Failure detection, determinism and resume on the GPU path: the device-side watchdog
(a reference medium too soft for the basic scheme diverges, as the oracle's iterates
do), the iteration cap, bitwise reproducibility of repeated solves (a missing
barrier in an LDS pass would show up as run-to-run differences), and resuming from a
checkpointed displacement."""
import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz
from oracle import tetra
from test_gpu_parity import SCHEMES, random_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _first_runaway(h, means):
    """First k where the watchdog fires on an oracle run: eps grown to 1e3 times its first
    value, or the residual norm L2 = eps ||<sigma>|| (strain loading) back above its first
    value and 10 times the smallest seen."""
    m = np.asarray(means)
    nrm = np.sqrt(m[:, 0] ** 2 + m[:, 1] ** 2 + m[:, 2] ** 2 + 2 * (m[:, 3] ** 2 + m[:, 4] ** 2 + m[:, 5] ** 2))
    L2 = np.asarray(h) * nrm
    best = L2[0]
    for k in range(1, len(h)):
        best = min(best, L2[k])
        if h[k] > 1e3 * h[0] or (L2[k] > L2[0] and L2[k] > 10 * best):
            return k
    return None


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_too_soft_reference_medium_is_reported_as_diverged(scheme):
    """lambda0 = 0.2 lambda_max: the iterates run away (the oracle's too); the watchdog
    stops the solve at the first iterate its rule flags, the same on both sides."""
    shape = (16, 16, 16)
    ph, C, _, E = random_problem(shape, 2, 60, "iso")
    s = np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5])
    top = max(np.linalg.eigvalsh(c * np.outer(s, s)).max() for c in C)
    C0 = syn.isotropic_voigt(0.2 * top, 0.0)
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    r = g.solve(E, C0=C0, tol=1e-10, max_iters=2000, trace=True, scheme=scheme)
    k = int(r.iters[0])
    ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=40, keep_fields=False)
    ko = _first_runaway(ref.history, ref.mean_history)
    _say(f"  diverged at iterate {k} (oracle history flags {ko}): residual {r.residual[0]:.3e}, "
         f"first {r.trace_residual[0, 0]:.3e}")
    assert r.rc == hz.HZ_EDIVERGED and r.status[0] == hz.HZ_EDIVERGED
    assert ko is not None and k == ko
    assert np.max(np.abs(r.trace_residual[0, : k + 1] - ref.history[: k + 1]) / ref.history[: k + 1]) < 1e-10


@pytest.mark.parametrize("contrast", [1e6, 1e8], ids=["c1e6", "c1e8"])
def test_stiff_inclusion_transient_is_not_flagged(contrast):
    """The contrast study's isolated sphere with a nearly rigid inclusion: eps rises by
    tens of times over the first iterates (<sigma> falls from the Voigt average) while the
    residual norm only decreases, and the scheme converges.  The FP64 solve to 1e-6 is not
    stopped by the watchdog and stops at the oracle's first iterate below 1e-6."""
    p = syn.isolated_sphere(contrast)
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    r = g.solve(p.loads, tol=1e-6, C0=p.C0, max_iters=2000, trace=True)
    k = int(r.iters[0])
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, p.loads[0], fixed_iters=k, keep_fields=False)
    k_o = int(np.argmax(ref.history < 1e-6))
    rise = ref.history.max() / ref.history[0]
    _say(f"  contrast {contrast:g}: stop iterate {k} (oracle {k_o}), eps rises {rise:.0f}x first")
    assert r.status[0] == hz.HZ_OK and k == k_o
    assert rise > 10 and _first_runaway(ref.history, ref.mean_history) is None


def test_iteration_cap_reports_not_converged():
    ph, C, C0, E = random_problem((12, 10, 8), 3, 61, "aniso")
    g = hz.Grid(12, 10, 8)
    g.set_material(C, ph)
    r = g.solve(E, C0=C0, tol=1e-14, max_iters=3, trace=True)
    assert r.rc == hz.HZ_NOT_CONVERGED and r.status[0] == hz.HZ_NOT_CONVERGED
    assert r.iters[0] == 3
    ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=3, keep_fields=False)
    assert abs(r.residual[0] - ref.history[3]) < 1e-10 * ref.history[3]
    assert np.abs(r.mean_sigma[0] - ref.mean_sigma).max() < 1e-12 * np.abs(ref.mean_sigma).max()


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_repeated_solves_are_bitwise_identical(scheme):
    """Fixed-order reductions and no atomics: two solves of the same loads give the
    same bits for every load, including the fields."""
    p = syn.boolean128(n=64, seed=7)
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    a = g.solve(p.loads[:3], C0=p.C0, fixed_iters=12, trace=True, fields=True, scheme=scheme)
    b = g.solve(p.loads[:3], C0=p.C0, fixed_iters=12, trace=True, fields=True, scheme=scheme)
    for name in ("mean_sigma", "trace_residual", "trace_mean", "eps", "sigma"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name


def _same(a, b, exact, name):
    if exact:
        assert np.array_equal(a, b), name
    else:
        scale = np.max(np.abs(b))
        assert np.max(np.abs(a - b)) <= 1e-11 * scale, (name, np.max(np.abs(a - b)) / scale)


@pytest.mark.parametrize("loading", [hz.HZ_LOAD_STRAIN, hz.HZ_LOAD_STRESS], ids=["strain", "stress"])
@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_resume_from_checkpoint(scheme, loading):
    """Checkpoint = the displacement of an iterate (and its mean strain under applied
    stress); a solve started from it continues the same iterates: bit for bit in the
    Fourier form; to rounding in the stencil form, whose iterate is held as its inverse
    z transform and converted to u(q) and back at the checkpoint."""
    shape = (16, 12, 10)
    ph, C, C0, E = random_problem(shape, 3, 62, "aniso")
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    if loading == hz.HZ_LOAD_STRESS:
        rng = np.random.default_rng(62)
        e0 = rng.normal(size=(3, 6)) * 5e-3
        e0[0] = 0.0
        g.set_eigenstrain(e0)
        E = np.array([[0.4, -0.1, 0.2, 0.05, -0.08, 0.12]])
    kw = dict(C0=C0, scheme=scheme, loading=loading)
    full = g.solve(E, fixed_iters=12, trace=True, fields=True, **kw)
    a = g.solve(E, fixed_iters=7, **kw)
    u7 = g.displacement(0)[None]
    b = g.solve(E, fixed_iters=5, trace=True, fields=True, u_init=u7, Ebar_init=a.Ebar, **kw)
    exact = scheme == hz.HZ_SCHEME_SPECTRAL
    _same(b.trace_residual[0, :6], full.trace_residual[0, 7:13], exact, "trace_residual")
    _same(b.trace_mean[0, :6], full.trace_mean[0, 7:13], exact, "trace_mean")
    for name in ("mean_sigma", "Ebar", "eps", "sigma"):
        _same(getattr(b, name), getattr(full, name), exact, name)


@pytest.mark.parametrize("shape", [(16, 8, 16), (8, 6, 4)], ids=["z16", "z4"])
def test_stencil_resume_with_single_pass_z_transforms(shape):
    """N3 = 16 and 4 are single radix passes, where the start-of-solve conversion of the
    given displacement runs in place with each thread owning whole z lines; two solves
    of 4 + 5 iterations continue the 9-iteration solve to rounding."""
    ph, C, C0, E = random_problem(shape, 2, 63, "iso")
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    if not g.scheme_available(hz.HZ_SCHEME_STENCIL):
        pytest.skip(f"stencil form not available for {shape}")
    kw = dict(C0=C0, scheme=hz.HZ_SCHEME_STENCIL)
    full = g.solve(E, fixed_iters=9, trace=True, fields=True, **kw)
    u9 = g.displacement(0)
    g.solve(E, fixed_iters=4, **kw)
    u4 = g.displacement(0)[None]
    b = g.solve(E, fixed_iters=5, trace=True, fields=True, u_init=u4, **kw)
    _same(b.trace_residual[0, :6], full.trace_residual[0, 4:10], False, "trace_residual")
    for name in ("mean_sigma", "eps", "sigma"):
        _same(getattr(b, name), getattr(full, name), False, name)
    _same(g.displacement(0), u9, False, "u")


@pytest.mark.parametrize("scheme", SCHEMES, ids=["spectral", "stencil"])
def test_refinement_falls_back_to_fp64_iterations(scheme):
    """Percolating stiff spheres (32^3, contrast 1e4): the FP32 corrections stop gaining
    far above tol, so the solve continues as plain FP64 iterations from U for the rest of
    its budget and reports HZ_FP64 as the path used; the reported residual is that of the
    reported displacement (an FP64 solve started from it measures the same eps_0)."""
    ph, _, _ = syn.boolean_spheres((32, 32, 32), 2.0, 0.3, 11)
    C = np.stack([syn.isotropic_voigt(1.0, 0.3), syn.isotropic_voigt(1e4, 0.3)])
    C0 = syn.ref_alpha_rule(1.0, 1e4, 0.3)
    g = hz.Grid(32, 32, 32)
    g.set_material(C, ph)
    E = np.array([syn.unit_load(0)])
    r = g.solve(E, C0=C0, tol=1e-8, precision=hz.HZ_FP32_REFINE, max_iters=3000, scheme=scheme)
    _say(f"  status {r.status[0]} path {r.precision_used[0]} iters {r.iters[0]} rounds {r.outer_rounds[0]} "
         f"residual {r.residual[0]:.3e}")
    assert r.precision_used[0] == hz.HZ_FP64
    assert r.status[0] in (hz.HZ_OK, hz.HZ_NOT_CONVERGED) and r.iters[0] <= 3000
    u = g.displacement(0)[None]
    chk = g.solve(E, C0=C0, fixed_iters=0, trace=True, u_init=u, scheme=scheme)
    assert abs(chk.trace_residual[0, 0] - r.residual[0]) <= 1e-9 * r.residual[0]
    assert np.abs(chk.mean_sigma[0] - r.mean_sigma[0]).max() <= 1e-9 * np.abs(r.mean_sigma[0]).max()

"""Solve server (continuous batching): a request's results in a mix of
requests on other grids, materials, shapes and precisions are bitwise those of
the same request served alone, and of the same loads through hz_solve; every
load keeps its own buffers, descriptor and device-side stop rule, so nothing
it computes depends on its neighbours or on when it was admitted."""
import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _grid(shape, seed, n_phases=2, aniso=False):
    rng = np.random.default_rng(seed)
    N1, N2, N3 = shape
    ph = rng.integers(0, n_phases, (N3, N2, N1)).astype(np.uint16)
    if aniso:
        C = np.stack([syn.random_spd_voigt(rng, 0.5, 8.0) for _ in range(n_phases)])
    else:
        C = np.stack([syn.isotropic_voigt(float(E), 0.3) for E in 10.0 ** rng.uniform(0, 1.5, n_phases)])
    g = hz.Grid(*shape)
    g.set_material(C, ph)
    return g


def _loads(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 6)) * 1e-3


# (grid key, shape, seed, aniso, n_loads, precision, tol, scheme)
AUTO, SPEC = hz.HZ_SCHEME_AUTO, hz.HZ_SCHEME_SPECTRAL
CASES = [
    ("a", (16, 16, 16), 1, False, 6, hz.HZ_FP64, 1e-8, AUTO),
    ("b", (12, 10, 8), 2, True, 2, hz.HZ_FP32_REFINE, 1e-8, AUTO),
    ("c", (16, 16, 16), 3, True, 3, hz.HZ_FP64, 1e-6, AUTO),       # same shape as a, other material
    ("d", (20, 12, 14), 4, False, 1, hz.HZ_FP32_REFINE, 1e-7, AUTO),
    ("a", (16, 16, 16), 1, False, 2, hz.HZ_FP32_REFINE, 1e-9, AUTO),  # same material as the first
    ("c", (16, 16, 16), 3, True, 2, hz.HZ_FP64, 1e-7, SPEC),       # the Fourier form beside the stencil form
]


def _make():
    grids = {}
    for key, shape, seed, aniso, *_ in CASES:
        if key not in grids:
            grids[key] = _grid(shape, seed, aniso=aniso)
    return grids


def _arena(grids, factor=1.2):
    total = 0
    for i, (key, _s, _seed, _a, nl, prec, _t, _sc) in enumerate(CASES):
        total += hz.request_bytes(grids[key], prec, nl)
    return int(total * factor)


def _alone(grids):
    out = []
    for i, (key, _s, _seed, _a, nl, prec, tol, sc) in enumerate(CASES):
        g = grids[key]
        srv = hz.Server(hz.request_bytes(g, prec, nl), max_problems=8)
        rid = srv.submit(g, _loads(nl, 100 + i), tol=tol, precision=prec, scheme=sc)
        srv.drain()
        r = srv.result(rid)
        assert r is not None and r.rc >= 0, r
        out.append(r)
    return out


def _same(a, b):
    return np.array_equal(a.mean_sigma, b.mean_sigma) and np.array_equal(a.iters, b.iters) and \
        np.array_equal(a.status, b.status) and np.array_equal(a.residual, b.residual)


@pytest.mark.parametrize("streams", [1, 3], ids=["one_stream", "three_streams"])
def test_mix_equals_alone_bitwise(streams):
    """streams = 3: the groups of a tick (three shapes, two precisions) spread over three
    streams and run on the device at the same time."""
    grids = _make()
    alone = _alone(grids)
    srv = hz.Server(_arena(grids), max_problems=32, check_every=4, streams=streams)
    ids = [srv.submit(grids[key], _loads(nl, 100 + i), tol=tol, precision=prec, scheme=sc)
           for i, (key, _s, _seed, _a, nl, prec, tol, sc) in enumerate(CASES)]
    srv.drain()
    for i, rid in enumerate(ids):
        r = srv.result(rid)
        _say(f"  case {i}: iters {r.iters} rounds {r.outer_rounds} res {r.residual}")
        assert _same(r, alone[i]), i
    # the same loads through hz_solve (same executor, one group) agree bitwise too
    for i, (key, _s, _seed, _a, nl, prec, tol, sc) in enumerate(CASES):
        rs = grids[key].solve(_loads(nl, 100 + i), tol=tol, precision=prec, scheme=sc)
        assert _same(rs, alone[i]), i
    # the two forms iterate the same scheme: same stop iterate, <sigma> equal to rounding
    E = _loads(2, 7)
    r_st = grids["c"].solve(E, tol=1e-9, scheme=hz.HZ_SCHEME_STENCIL)
    r_sp = grids["c"].solve(E, tol=1e-9, scheme=hz.HZ_SCHEME_SPECTRAL)
    assert np.array_equal(r_st.iters, r_sp.iters)
    assert np.abs(r_st.mean_sigma - r_sp.mean_sigma).max() < 1e-12 * np.abs(r_sp.mean_sigma).max()


def test_continuous_arrivals_and_admission_under_memory_pressure():
    """Requests arrive while others run; the arena holds only about two requests,
    so later ones wait in the queue and are admitted as memory frees up."""
    grids = _make()
    alone = _alone(grids)
    biggest = max(hz.request_bytes(grids[k], p, n) for k, _s, _sd, _a, n, p, _t, _sc in CASES)
    srv = hz.Server(int(2.05 * biggest), max_problems=16, check_every=2, streams=2)
    ids = {}
    saw_queue = False
    pending = list(range(len(CASES)))
    tick = 0
    while pending or any(srv.pending()):
        if pending and tick % 3 == 0:  # one arrival every third tick
            i = pending.pop(0)
            key, _s, _sd, _a, nl, prec, tol, sc = CASES[i]
            ids[i] = srv.submit(grids[key], _loads(nl, 100 + i), tol=tol, precision=prec, scheme=sc)
        q, _r = srv.pending()
        saw_queue |= q > 0
        srv.step()
        tick += 1
        assert tick < 100000
    assert saw_queue
    for i, rid in ids.items():
        r = srv.result(rid)
        assert r is not None and _same(r, alone[i]), i
        assert np.all(r.wall_seconds > 0)


def test_release_of_queued_request_and_errors():
    g = _grid((8, 8, 8), 9)
    need = hz.request_bytes(g, hz.HZ_FP64, 1)
    srv = hz.Server(need, max_problems=4, check_every=1)
    a = srv.submit(g, _loads(1, 1), tol=1e-6)
    b = srv.submit(g, _loads(1, 2), tol=1e-6)  # waits: the arena fits one request
    srv.step()
    q, r = srv.pending()
    assert q == 1 and r == 1
    assert hz.lib().hz_server_release(srv._h, b) == 0  # withdraw the queued one
    assert hz.lib().hz_server_release(srv._h, a) == hz._abi.HZ_EINVAL  # running
    srv.drain()
    assert srv.result(a).rc >= 0
    with pytest.raises(hz.HzError) as e:
        srv.submit(g, _loads(2, 3), tol=1e-6)  # two loads never fit
    assert e.value.code == hz._abi.HZ_EWORKSPACE
    for bad in (0, 9):
        assert hz.lib().hz_server_set_streams(srv._h, bad) == hz._abi.HZ_EINVAL


KINDS = [("iso", False, False), ("iso_eig", False, True), ("aniso", True, False), ("aniso_eig", True, True)]


@pytest.mark.parametrize("shape", [(16, 12, 10), (14, 10, 12)], ids=["n1_16", "n1_14"])
def test_served_requests_match_the_oracle_for_every_material_kind(shape):
    """One FP64 and one FP32+refine request per material kind (isotropic or anisotropic
    phases, with or without eigenstrains), served together in one mix.  FP64: <sigma> and
    the residual at the served stop iterate against the oracle run to that iterate
    (<= 1e-10 relative).  FP32+refine: <sigma> within 1e-6 of the converged oracle.
    N1 = 14 serves a grid whose stencil-form x transforms run in one radix-7 pass."""
    from oracle import tetra

    grids, probs = [], []
    for i, (name, aniso, eig) in enumerate(KINDS):
        rng = np.random.default_rng(300 + i)
        N1, N2, N3 = shape
        ph = rng.integers(0, 3, (N3, N2, N1)).astype(np.uint16)
        if aniso:
            C = np.stack([syn.random_spd_voigt(rng, 0.5, 8.0) for _ in range(3)])
        else:
            C = np.stack([syn.isotropic_voigt(float(E), 0.3) for E in 10.0 ** rng.uniform(0, 1.5, 3)])
        s = np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5])
        C0 = syn.isotropic_voigt(0.75 * max(np.linalg.eigvalsh(c * np.outer(s, s)).max() for c in C), 0.0)
        e0 = rng.normal(size=(3, 6)) * 2e-3 if eig else None
        g = hz.Grid(*shape)
        g.set_material(C, ph)
        if eig:
            g.set_eigenstrain(e0)
        grids.append(g)
        probs.append((ph, C, C0, e0, _loads(1, 400 + i)))
    need = sum(hz.request_bytes(g, p, 1) for g in grids for p in (hz.HZ_FP64, hz.HZ_FP32_REFINE))
    srv = hz.Server(int(1.2 * need), max_problems=16, check_every=4)
    ids = []
    for g, (ph, C, C0, e0, E) in zip(grids, probs):
        ids.append((srv.submit(g, E, tol=1e-8, C0=C0, precision=hz.HZ_FP64),
                    srv.submit(g, E, tol=1e-8, C0=C0, precision=hz.HZ_FP32_REFINE)))
    srv.drain()
    for (name, _a, _e), (i64, i32), (ph, C, C0, e0, E) in zip(KINDS, ids, probs):
        r64 = srv.result(i64)
        r32 = srv.result(i32)
        assert r64.status[0] == hz.HZ_OK and r32.status[0] == hz.HZ_OK, name
        k = int(r64.iters[0])
        ref = tetra.basic_scheme(ph, C, C0, E[0], fixed_iters=k, eps0=e0, keep_fields=False)
        scale = np.abs(ref.mean_sigma).max()
        em = np.abs(r64.mean_sigma[0] - ref.mean_sigma).max() / scale
        # the residual of a converged iterate is a norm of r(q), a difference of terms of
        # the size of the stress: rounding is measured against the first residual's scale
        eh = abs(r64.residual[0] - ref.history[k]) / ref.history[0]
        conv = tetra.basic_scheme(ph, C, C0, E[0], tol=1e-12, eps0=e0, keep_fields=False)
        e32 = np.abs(r32.mean_sigma[0] - conv.mean_sigma).max() / np.abs(conv.mean_sigma).max()
        _say(f"  served {name}: FP64 stop iterate {k} (oracle first below tol: "
             f"{int(np.argmax(ref.history < 1e-8)) if (ref.history < 1e-8).any() else None}), "
             f"<sigma> {em:.1e}, residual {eh:.1e}; FP32+refine vs converged {e32:.1e}")
        assert ref.history[k] < 1e-8 and (k == 0 or ref.history[k - 1] >= 1e-8 * (1 - 1e-9))
        assert em < 1e-10 and eh < 1e-10
        assert e32 < 1e-6

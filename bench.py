#!/usr/bin/env python3
"""Benchmark of the tetrahedral-stencil basic scheme on one MI355X.

Workload (the headline configuration): 128^3 periodic cell, Boolean model of
overlapping spheres (radius 8, seeded, 30% volume fraction), stiffness
contrast 1e3 (nu = 0.3), all six unit macroscopic strains solved as one batch
in FP64 (the effective-stiffness computation).  A "step" is one iteration of
Algorithm 1 over all six loads.  The default realisation is the stencil form
(transforms of the 3 displacement components, real-space strains, constitutive
law and corner forces, transforms of the 3 force components, Green-operator
update, FP64 residual reduction); the Fourier form (12 strain/stress fields
through the transforms) is timed beside it for context.

Prints ONE JSON line:
  value          voxel-iterations/s (128^3 voxels x 6 loads x steps / timed seconds)
  roofline       the dominant kernel's algorithmic bytes per launch / its mean
                 HIP-event duration over the timed iterations (events around that
                 kernel's launches only), against 8 TB/s
  per_kernel     mean launch durations from an untimed run with events around every
                 launch (it also picks the dominant kernel)
  iteration_roofline_frac  the whole iteration's algorithmic bytes per voxel-iteration
                 x value / 8 TB/s
  ceff_converged the same workload run to eps < 1e-8 (FP64, and FP32+refine beside it):
                 C_eff, iterations and status per load, symmetry residual, the margins to
                 the Voigt and Reuss bounds
  full_size      FP64 fixed-iteration throughput and whole-iteration roofline fraction of
                 the 256^3 Voronoi polycrystal and of the 192x192x320 Boolean spheres (6
                 loads each), with per-kernel rates, and the FP32 iteration (fixed FP32
                 count) on the same workloads
  cpu_baseline   the CPU oracle timed on the host on a bounded sample (CPU model stated)
  time_to_1e-6   FP32+refinement vs plain FP64 device time to an FP64-verified
                 residual of 1e-6 on the 256^3 Voronoi polycrystal (6 loads); the speedup
                 only when every load of both solves converged
  green_operators  the comparison Green operators of Sec. 3.2 / Appendix B (rotated,
                 continuous-frequency) beside the tetrahedral scheme: the 64^3 cubic void
                 under 300 MPa (iterates to 1e-4/1e-6/1e-10, artefact measures of the
                 stress field) and the FP64 iteration rate of each on the headline workload
  serving        a seeded stream of solve requests (grid sizes 32..192^3, Boolean
                 spheres or cubic polycrystals, contrast log-uniform 1e1..1e6, one
                 load each, FP32+refine to 1e-6) through the solve server: closed-loop
                 saturation throughput, then Poisson arrivals at 0.7x that rate with
                 p50/p99 latency from arrival to result over the requests that reached
                 1e-6, the count of those that did not beside them
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "voxel-iters/s + time-to-1e-6 residual, FP32+refine vs FP64; p50/p99 solve latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2405_11168_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bytes(kind, S, N, nloads, csz):
    """Algorithmic HBM bytes of one launch of a pass over `nloads` problems: complex
    spectra (S complex elements per field, csz bytes each) and real fields (N values,
    csz/2 bytes each) each read or written once, plus the uint16 phase map."""
    rsz = csz // 2
    spectral = {                         # Fourier form: 12 strain/stress fields
        "zexpand": 15 * S * csz,         # read u (3), write 12 strain spectra
        "yinv": 24 * S * csz,            # read 12, write 12
        "yfwd": 24 * S * csz,
        "xpass": 24 * S * csz + 2 * N,   # read 12, write 12, phase map
        "zcontract": 18 * S * csz,       # read 12 stress spectra + u, write u
    }
    stencil = {                          # stencil form: 3 displacement / force fields
        "zconvert3": 6 * S * csz,        # u(q) <-> mixed domain in place (once per solve)
        "yinv3": 6 * S * csz,            # read the mixed-domain u, write 3 fields
        "xc2r": 3 * S * csz + 3 * N * rsz,
        "stencil": 6 * N * rsz + 2 * N,  # read u (corners), write g, phase map
        "xr2c": 3 * N * rsz + 3 * S * csz,
        "yfwd3": 6 * S * csz,
        "zcontract3": 9 * S * csz,       # read g and the mixed-domain u, write u
    }
    table = {**spectral, **stencil}
    if kind not in table:
        return None
    return table[kind] * nloads


def iteration_bytes(scheme, S, N, csz):
    """Algorithmic bytes of one iteration of one load (sum over its passes)."""
    kinds = (["zexpand", "yinv", "xpass", "yfwd", "zcontract"] if scheme == "spectral" else
             ["yinv3", "xc2r", "stencil", "xr2c", "yfwd3", "zcontract3"])
    return sum(kernel_bytes(k, S, N, 1, csz) for k in kinds)


def host_cpu():
    """CPU model name and the logical CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(problem, max_seconds=20.0):
    """The oracle (FP64 numpy/scipy, Algorithm 1) on a bounded sample: one load,
    a few iterations of the same 128^3 workload, timed on the host."""
    from oracle import tetra

    n = problem.phase.size
    iters = 1
    t0 = time.perf_counter()
    tetra.basic_scheme(problem.phase, problem.C, problem.C0, problem.loads[0], fixed_iters=iters - 1,
                       keep_fields=False)
    dt = time.perf_counter() - t0
    k = max(1, min(16, int(max_seconds / max(dt, 1e-3))))
    if k > 1:
        t0 = time.perf_counter()
        tetra.basic_scheme(problem.phase, problem.C, problem.C0, problem.loads[0], fixed_iters=k - 1,
                           keep_fields=False)
        dt = time.perf_counter() - t0
        iters = k
    model, avail = host_cpu()
    return {"value": n * iters / dt, "unit": "voxel-iters/s", "cores": tetra.WORKERS, "kind": "oracle",
            "cpu_model": model, "cpus_available": avail,
            "sample": f"1 of 6 loads, {iters} iteration(s) of the 128^3 workload (FP64 numpy+scipy.fft, "
                      f"{tetra.WORKERS} FFT threads), {dt:.1f} s wall"}


def time_to_tol(hz, np, torch, p, g):
    """Device time to an FP64-verified residual of 1e-6 on the periodic Voronoi
    polycrystal (200 cubic grains C11=168, C12=121, C44=75, random orientations,
    6 unit loads): plain FP64 iterations against FP32 iterations anchored by FP64
    sweeps.  Each variant runs three times: a warmup, a run with HIP events around
    every launch (per-kernel times), and the reported run without them.  The speedup
    is reported only when every load of both solves converged."""
    n = p.shape[0]
    out = {"workload": f"voronoi{n}_200grains_cubic_6loads", "tol": 1e-6}
    res = {}
    for prec, name in ((hz.HZ_FP64, "fp64"), (hz.HZ_FP32_REFINE, "fp32_refine")):
        g.bind(prec, 6)
        for rep in range(3):
            g.profile(rep == 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.solve(p.loads, C0=p.C0, tol=1e-6, precision=prec, check_every=4)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if rep == 1:
                prof = g.profile_read()
        g.profile(False)
        res[name] = r
        ok = bool(np.all(r.status == hz.HZ_OK) and np.all(r.seconds_to_1e6 > 0))
        out[name] = {"all_converged": ok, "status": [int(x) for x in r.status],
                     "seconds_to_1e-6": round(float(np.max(r.seconds_to_1e6)), 4) if ok else None,
                     "wall_s": round(wall, 4), "iters": [int(x) for x in r.iters],
                     "outer_rounds": [int(x) for x in r.outer_rounds], "residual": float(np.max(r.residual)),
                     "kernel_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in prof.items()}}
    both = out["fp64"]["all_converged"] and out["fp32_refine"]["all_converged"]
    out["speedup"] = (round(out["fp64"]["seconds_to_1e-6"] / out["fp32_refine"]["seconds_to_1e-6"], 3)
                      if both else None)
    m64, m32 = res["fp64"].mean_sigma, res["fp32_refine"].mean_sigma
    out["ceff_rel_diff_fp32r_vs_fp64"] = float(np.abs(m32 - m64).max() / np.abs(m64).max())
    return out


def kernel_rates(prof, S, N, nloads):
    """Per kernel of a profiled run: mean ms per launch and, where the kernel has an
    algorithmic byte count (launches over all `nloads` loads; the stencil-state
    conversion runs per load), its achieved GB/s and fraction of 8 TB/s."""
    out = {}
    for name, (ms, cnt) in sorted(prof.items()):
        kind, prec = name.rsplit("_", 1)
        b = kernel_bytes(kind, S, N, 1 if kind == "zconvert3" else nloads, 16 if prec == "f64" else 8)
        t = ms / cnt
        e = {"ms_per_launch": round(t, 4), "launches": cnt}
        if b is not None:
            gbs = b / (t * 1e-3) / 1e9
            e.update({"GB_per_launch": round(b / 1e9, 4), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        out[name] = e
    return out


def full_size_leg(hz, np, torch, name, p, g, loads, K1=4, K2=24):
    """Iteration rate of `loads` on one full-size grid, FP64 and FP32, from two runs of
    fixed length: (t(K2) - t(K1)) / (K2 - K1) per iteration, so the solve's set-up and
    its final measurement cancel.  FP32: a fixed FP32 count (K FP32 updates, one FP64
    sweep).  A third, profiled run of K2 gives the per-kernel rates."""
    N1, N2, N3 = p.shape
    N = N1 * N2 * N3
    S = (N1 // 2 + 1) * N2 * N3
    nl = len(loads)
    out = {"workload": name, "grid": [N1, N2, N3], "loads": nl, "passes_timed": K2 - K1}
    for prec, key, csz in ((hz.HZ_FP64, "fp64", 16), (hz.HZ_FP32_REFINE, "fp32", 8)):
        g.bind(prec, nl)

        def run(K):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.solve(loads, C0=p.C0, precision=prec, fixed_iters=K, check_every=1 << 20)
            torch.cuda.synchronize()
            assert np.all(r.iters == K), r.iters
            return time.perf_counter() - t0

        run(2)
        t1, t2 = run(K1), run(K2)
        g.profile(True)
        run(K2)
        torch.cuda.synchronize()
        g.profile(False)
        prof = g.profile_read()
        per_iter = (t2 - t1) / (K2 - K1)
        scheme = "stencil" if any(k.startswith("stencil") for k in prof) else "spectral"
        bpv = iteration_bytes(scheme, S, N, csz) / N
        vips = N * nl / per_iter
        out[key] = {"ms_per_iteration": round(per_iter * 1e3, 4), "voxel_iters_per_s": vips, "scheme": scheme,
                    "bytes_per_voxel_iteration": round(bpv, 1),
                    "iteration_roofline_frac": round(vips * bpv / (HBM_PEAK_GBS * 1e9), 4),
                    "kernels": {k: v for k, v in kernel_rates(prof, S, N, nl).items()
                                if k.endswith("f64" if key == "fp64" else "f32")}}
    return out


def compare_leg(syn, hz, np, torch, K1=4, K2=24, parts=("void", "hard", "contrast", "rates")):
    """The comparison Green operators of Sec. 3.2 and Appendix B beside the tetrahedral
    scheme (FP64; the comparison operators run in the spectral form).

    (1) The cubic void of Sec. 3.2 at the paper's size: a 31^3 void in a 64^3 cell
    (mu = 132.30 GPa, nu = 0.26), hydrostatic pressure 300 MPa as an applied stress,
    lambda0 = 0.8 lambda_m, run to eps < 1e-10 (cap 4000 iterates, traced): iterates to
    1e-4, 1e-6 and 1e-10, device seconds, and two measures of the artefacts the paper
    shows in its stress maps, taken on the stress field of the reported iterate:
    'checkerboard_frac', the share of the stress field's spectral energy (q != 0) on
    the lines where two components of q equal pi (the rotated scheme's zero set), and
    'line_osc_MPa', the largest second difference of sigma_11 along the (100) line
    through the void centre, over matrix voxels at least two voxels from a void face.
    (2) The hard sphere of Sec. 3.3 and (3) iterates against contrast for the isolated
    sphere of Sec. 3.4 (hard_sphere_compare, contrast_compare).
    (4) The iteration rate of each operator on the headline workload (128^3 Boolean
    spheres, contrast 1e3, 6 loads), from two fixed-length runs, with per-kernel rates."""
    out = {}
    ops = (("tetra_stencil", hz.HZ_GREEN_TETRA, hz.HZ_SCHEME_STENCIL),
           ("tetra_spectral", hz.HZ_GREEN_TETRA, hz.HZ_SCHEME_SPECTRAL),
           ("rotated", hz.HZ_GREEN_ROTATED, hz.HZ_SCHEME_AUTO),
           ("continuous", hz.HZ_GREEN_CONTINUOUS, hz.HZ_SCHEME_AUTO))
    if "void" in parts:
        out["cubic_void"] = cubic_void_compare(syn, hz, np, ops)
    if "hard" in parts:
        out["hard_sphere"] = hard_sphere_compare(syn, hz, np, ops)
    if "contrast" in parts:
        out["contrast"] = contrast_compare(syn, hz, np, ops)
    if "rates" in parts:
        out["iteration_rate"] = compare_rates(syn, hz, np, torch, ops, K1, K2)
    return out


def von_mises(np, s):
    """von Mises stress of a field of tensor comps (11,22,33,23,13,12) on axis 0."""
    d = 0.5 * ((s[0] - s[1]) ** 2 + (s[1] - s[2]) ** 2 + (s[2] - s[0]) ** 2)
    return np.sqrt(d + 3.0 * (s[3] ** 2 + s[4] ** 2 + s[5] ** 2))


def hard_sphere_compare(syn, hz, np, ops):
    """Sec. 3.3: the glass sphere in polyamide (128^3, R = 40, eps_11 = 0.05, lambda0 the mean
    of the two stiffnesses) with each operator, the tetrahedral and rotated ones to 1e-10, the
    continuous one to 1e-4 as in the paper (cap 4000 iterates): iterates, and the largest
    second difference of the von Mises stress along the (100) line through the centre, in
    the matrix and in the inclusion, over voxels at least two voxels from the interface."""
    p = syn.hard_sphere()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    n = p.shape[0]
    line = p.phase[n // 2, n // 2, :]
    inside = line == 1
    x = np.arange(n)
    edge = np.nonzero(np.diff(line.astype(int)) != 0)[0]
    far = np.ones(n, dtype=bool)
    for e in edge:
        far &= np.abs(x - e - 0.5) > 2.5
    out = {"workload": "glass sphere R = 40 in a 128^3 polyamide cell, eps_11 = 0.05", "vf": p.info["vf"]}
    for name, green, scheme in ops:
        if name == "tetra_spectral":
            continue
        tol = 1e-4 if green == hz.HZ_GREEN_CONTINUOUS else 1e-10
        r = g.solve(p.loads, C0=p.C0, tol=tol, max_iters=4000, fields=True, scheme=scheme, green=green)
        vm = von_mises(np, r.sigma[0][:, n // 2, n // 2, :])
        d2 = np.abs(np.roll(vm, -1) - 2 * vm + np.roll(vm, 1))
        out[name] = {"status": int(r.status[0]), "tol": tol, "iters": int(r.iters[0]),
                     "residual": float(r.residual[0]), "C11_eff": round(float(r.mean_sigma[0][0]) / 0.05, 3),
                     "vm_osc_matrix_MPa": round(float(d2[far & ~inside].max()), 3),
                     "vm_osc_inclusion_MPa": round(float(d2[far & inside].max()), 3)}
        log(f"bench: compare hard sphere {name}: {out[name]}")
    return out


def contrast_compare(syn, hz, np, ops, contrasts=(1e-2, 1e-1, 10.0, 1e2, 1e3, 1e4), cap=20000):
    """Sec. 3.4: iterates to eps < 1e-10 of the isolated sphere against the bulk-modulus
    contrast, for each operator (cap 20000).  The paper's 44^3 cell has a factor 11 the
    transforms do not take; 42^3 with the same radius ratio (R = 0.4 N = 16.8) stands in,
    nu = 0.125, alpha-rule reference."""
    out = {"workload": "isolated sphere 42^3, R = 16.8, nu = 0.125, tol 1e-10", "cap": cap,
           "contrasts": list(contrasts)}
    for name, green, scheme in ops:
        if name == "tetra_spectral":
            continue
        row = []
        for c in contrasts:
            p = syn.isolated_sphere(c, n=42)
            g = hz.Grid(*p.shape)
            g.set_material(p.C, p.phase)
            r = g.solve(p.loads, C0=p.C0, tol=1e-10, max_iters=cap, scheme=scheme, green=green)
            row.append(int(r.iters[0]) if r.status[0] == hz.HZ_OK else
                       f"{int(r.iters[0])} (eps {float(r.residual[0]):.1e}, status {int(r.status[0])})")
        out[name] = row
        log(f"bench: compare contrast {name}: {row}")
    return out


def cubic_void_compare(syn, hz, np, ops):
    N = 64
    ph = np.zeros((N, N, N), dtype=np.uint16)
    ph[16:47, 16:47, 16:47] = 1
    mu, nu = 132.30e3, 0.26
    Cm = syn.isotropic_voigt(2.0 * mu * (1.0 + nu), nu)
    C = np.stack([Cm, np.zeros((6, 6))])
    sa = np.array([[-300.0, -300.0, -300.0, 0.0, 0.0, 0.0]])
    g = hz.Grid(N, N, N)
    g.set_material(C, ph)
    h = np.arange(N)
    lines = (((2 * h == N)[:, None, None].astype(int) + (2 * h == N)[None, :, None]
              + (2 * h == N)[None, None, :]) >= 2)
    lines[0, 0, 0] = False
    x = np.arange(N)
    matrix = (x < 16 - 2) | (x > 46 + 2)
    void = {"workload": "cubic void 31^3 in 64^3, P = 300 MPa, lambda0 = 0.8 lambda_m", "tol": 1e-10, "cap": 4000}
    for name, green, scheme in ops:
        r = g.solve(sa, C0=0.8 * Cm, tol=1e-10, max_iters=4000, loading=hz.HZ_LOAD_STRESS, fields=True,
                    trace=True, scheme=scheme, green=green)
        tr = r.trace_residual[0]
        tr = tr[np.isfinite(tr)]

        def first(t):
            k = np.nonzero(tr < t)[0]
            return int(k[0]) if k.size else None

        sig = r.sigma[0]
        spec = np.fft.fftn(sig, axes=(1, 2, 3))
        e = np.sum(np.abs(spec) ** 2, axis=0)
        e[0, 0, 0] = 0.0
        s11 = sig[0, 31, 31, :]
        d2 = np.abs(np.roll(s11, -1) - 2 * s11 + np.roll(s11, 1))
        void[name] = {"status": int(r.status[0]), "iters": int(r.iters[0]), "residual": float(r.residual[0]),
                      "iters_to_1e-4": first(1e-4), "iters_to_1e-6": first(1e-6), "iters_to_1e-10": first(1e-10),
                      "seconds": round(float(r.seconds[0]), 4),
                      "checkerboard_frac": float(e[lines].sum() / e.sum()),
                      "line_osc_MPa": round(float(d2[matrix].max()), 4),
                      "mean_sigma": [round(float(v), 6) for v in r.mean_sigma[0][:3]]}
        log(f"bench: compare cubic void {name}: {void[name]}")
    return void


def compare_rates(syn, hz, np, torch, ops, K1, K2):
    p = syn.boolean128()
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    g.bind(hz.HZ_FP64, 6)
    N1, N2, N3 = p.shape
    Nv, S = N1 * N2 * N3, (N1 // 2 + 1) * N2 * N3
    rates = {"workload": "boolean128_c1e3_6loads", "passes_timed": K2 - K1}
    for name, green, scheme in ops:
        def run(K):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.solve(p.loads, C0=p.C0, fixed_iters=K, check_every=1 << 20, scheme=scheme, green=green)
            torch.cuda.synchronize()
            assert np.all(r.iters == K), r.iters
            return time.perf_counter() - t0

        run(2)
        t1, t2 = run(K1), run(K2)
        g.profile(True)
        run(K2)
        torch.cuda.synchronize()
        g.profile(False)
        prof = g.profile_read()
        per_iter = (t2 - t1) / (K2 - K1)
        form = "stencil" if scheme == hz.HZ_SCHEME_STENCIL else "spectral"
        bpv = iteration_bytes(form, S, Nv, 16) / Nv
        vips = Nv * 6 / per_iter
        rates[name] = {"ms_per_iteration": round(per_iter * 1e3, 4), "voxel_iters_per_s": vips,
                       "bytes_per_voxel_iteration": round(bpv, 1),
                       "iteration_roofline_frac": round(vips * bpv / (HBM_PEAK_GBS * 1e9), 4),
                       "kernels": kernel_rates(prof, S, Nv, 6)}
        log(f"bench: compare rate {name}: {per_iter * 1e3:.3f} ms per 6-load iteration, {vips / 1e9:.2f} G")
    return rates


def bounds_margins(np, Ce, C, phase):
    """Symmetry residual of C_eff and its margins to the Voigt bound (volume average of
    the stiffnesses) and the Reuss bound (inverse of the average compliance): the
    smallest eigenvalue of C_V - C_eff and of C_eff - C_R in Mandel form (shear rows and
    columns of the engineering-shear Voigt matrix scaled by sqrt 2), relative to the largest eigenvalue of C_eff; both are
    >= 0 for an admissible result."""
    f = np.bincount(phase.ravel(), minlength=len(C)) / phase.size
    CV = np.einsum("p,pij->ij", f, C)
    if any(fp > 0 and not np.any(c) for fp, c in zip(f, C)):
        CR = np.zeros((6, 6))  # a void phase: infinite average compliance, the Reuss bound is 0
    else:
        CR = np.linalg.inv(np.einsum("p,pij->ij", f, np.linalg.inv(C)))
    W = np.diag(np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5]))  # Mandel = W C W for engineering-shear Voigt
    sym = 0.5 * (Ce + Ce.T)
    top = np.linalg.eigvalsh(W @ sym @ W).max()
    return {"symmetry_residual": float(np.abs(Ce - Ce.T).max() / np.abs(Ce).max()),
            "voigt_margin": float(np.linalg.eigvalsh(W @ (CV - sym) @ W).min() / top),
            "reuss_margin": float(np.linalg.eigvalsh(W @ (sym - CR) @ W).min() / top)}


def ceff_leg(hz, np, torch, p, g, tol=1e-8, max_iters=200000):
    """C_eff of the headline workload run to convergence: the six unit loads as one
    batch (hz_effective_stiffness), FP64 and FP32+refine."""
    out = {"workload": "boolean128_contrast1e3_6loads", "tol": tol, "max_iters": max_iters}
    res = {}
    for prec, key in ((hz.HZ_FP64, "fp64"), (hz.HZ_FP32_REFINE, "fp32_refine")):
        g.bind(prec, 6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ce, r = g.effective_stiffness(tol=tol, max_iters=max_iters, precision=prec, C0=p.C0, check_every=64)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[key] = Ce
        out[key] = {"all_converged": bool(np.all(r.status == hz.HZ_OK)), "status": [int(x) for x in r.status],
                    "iters": [int(x) for x in r.iters], "outer_rounds": [int(x) for x in r.outer_rounds],
                    "residual": [float(x) for x in r.residual], "device_s": round(float(np.max(r.seconds)), 3),
                    "wall_s": round(wall, 3), "C_eff": [[float(f"{x:.9g}") for x in row] for row in Ce],
                    **bounds_margins(np, Ce, p.C, p.phase)}
    out["ceff_rel_diff_fp32r_vs_fp64"] = float(np.abs(res["fp32_refine"] - res["fp64"]).max() /
                                               np.abs(res["fp64"]).max())
    return out


def sweep_leg(syn, hz, np, torch, grids, contrasts, cap=40000, stiff_budget=4000):
    """The contrast sweep on Boolean spheres (R = 8 to vf 0.25, seed 4; matrix E = 1,
    nu = 0.3; alpha-rule lambda0), load E_xx to tol 1e-6 in FP64 and FP32+refine.
    Contrasts that converge run to tol under a large cap; stiff ones (C >= 1e4) run a
    traced budget and report the residual reached and its decay over the last 1000
    iterations.  At the converging endpoints (voids and C = 10) all six loads solve as
    one batch and C_eff is reported with its symmetry and bound margins."""
    rows, ends = [], []
    for shape in grids:
        for C in contrasts:
            p = syn.sphere_contrast(shape, C)
            g = hz.Grid(*shape)
            g.set_material(p.C, p.phase)
            row = {"grid": list(shape), "contrast": C, "n_spheres": p.info["n_spheres"], "vf": round(p.info["vf"], 4)}
            stiff = C >= 1e4
            for prec, key in ((hz.HZ_FP64, "fp64"), (hz.HZ_FP32_REFINE, "fp32_refine")):
                g.bind(prec, 1)
                torch.cuda.synchronize()
                r = g.solve(p.loads, tol=1e-6, max_iters=stiff_budget if stiff else cap, precision=prec, C0=p.C0,
                            trace=stiff, check_every=64)
                torch.cuda.synchronize()
                e = {"status": int(r.status[0]), "iters": int(r.iters[0]), "fp64_sweeps": int(r.outer_rounds[0]),
                     "residual": float(r.residual[0]), "device_s": round(float(r.seconds[0]), 4),
                     "seconds_to_1e-6": round(float(r.seconds_to_1e6[0]), 4)}
                if stiff:
                    h = np.asarray(r.trace_residual[0])
                    h = h[np.isfinite(h) & (h > 0)]
                    if len(h) > 1200:
                        slope = np.polyfit(np.arange(1000), np.log10(h[-1000:]), 1)[0]
                        e["iters_per_decade_last_1000"] = round(-1.0 / slope, 1) if slope < 0 else None
                row[key] = e
            log(f"bench: sweep {row}")
            rows.append(row)
            if C in (0.0, 10.0):
                end = {"grid": list(shape), "contrast": C}
                res = {}
                for prec, key in ((hz.HZ_FP64, "fp64"), (hz.HZ_FP32_REFINE, "fp32_refine")):
                    g.bind(prec, 6)
                    Ce, r6 = g.effective_stiffness(tol=1e-6, max_iters=cap, precision=prec, C0=p.C0, check_every=64)
                    torch.cuda.synchronize()
                    res[key] = Ce
                    end[key] = {"all_converged": bool(np.all(r6.status == hz.HZ_OK)),
                                "iters": [int(x) for x in r6.iters], "device_s": round(float(np.max(r6.seconds)), 3),
                                "C_eff": [[float(f"{x:.7g}") for x in row_] for row_ in Ce],
                                **bounds_margins(np, Ce, p.C, p.phase)}
                end["ceff_rel_diff_fp32r_vs_fp64"] = float(np.abs(res["fp32_refine"] - res["fp64"]).max() /
                                                           np.abs(res["fp64"]).max())
                log(f"bench: sweep endpoint {end}")
                ends.append(end)
            del g
            torch.cuda.empty_cache()
    # the isolated inclusion of the contrast study: FP64 iterations to 1e-10, and to 1e-6 in
    # FP64 and FP32+refine where FP64 rounding floors the residual above 1e-10
    iso_rows = []
    for C in (0.0, 1e-6, 1e-3, 0.1, 10.0, 1e2, 1e3, 1e4, 1e6, 1e8):
        p = syn.isolated_sphere(C)
        g = hz.Grid(*p.shape)
        g.set_material(p.C, p.phase)
        row = {"contrast": C, "vf": round(p.info["vf"], 4)}
        for prec, tol, key in ((hz.HZ_FP64, 1e-10, "fp64_1e-10"), (hz.HZ_FP64, 1e-6, "fp64_1e-6"),
                               (hz.HZ_FP32_REFINE, 1e-6, "fp32_refine_1e-6")):
            g.bind(prec, 1)
            r = g.solve(p.loads, tol=tol, max_iters=20000, precision=prec, C0=p.C0, check_every=16)
            row[key] = {"status": int(r.status[0]), "iters": int(r.iters[0]), "residual": float(r.residual[0])}
        log(f"bench: sweep isolated {row}")
        iso_rows.append(row)
        del g
    return {"workload": "Boolean spheres R 8 to vf 0.25 (seed 4), matrix E 1 nu 0.3, alpha-rule lambda0, "
                        "E_xx to tol 1e-6; six loads at C = 0 and 10; the isolated sphere of hz_synth.isolated_sphere "
                        "(48^3, R = 0.4 N, nu 0.125)",
            "rows": rows, "endpoints": ends, "isolated": iso_rows}


def serving_leg(syn, hz, np, torch, n_req, max_iters, load_factors=(0.7,), seed=5, streams=1):
    """Closed loop (all requests at t=0) for the saturation rate, then an open
    loop with Poisson arrivals at load_factor x that rate.  Latency = result
    ready (the server step that retired the request) - arrival time."""
    t0 = time.perf_counter()
    reqs, grids = [], []
    for i in range(n_req):
        p = syn.serving_request(i)
        g = hz.Grid(*p.shape)
        g.set_material(p.C, p.phase)
        reqs.append(p)
        grids.append(g)
        if (i + 1) % 250 == 0:
            print(f"serve: {i + 1} of {n_req} requests generated", file=sys.stderr, flush=True)
    gen_s = time.perf_counter() - t0
    need = [hz.request_bytes(g, hz.HZ_FP32_REFINE, 1) for g in grids]
    arena = min(int(1.05 * sum(need)), 160 << 30)
    srv = hz.Server(arena, max_problems=n_req + 8, check_every=8, streams=streams)

    def submit(i):
        p = reqs[i]
        return srv.submit(grids[i], p.loads, tol=1e-6, precision=hz.HZ_FP32_REFINE, C0=p.C0, max_iters=max_iters)

    # warm the kernels of every shape once (untimed)
    seen = {}
    for i, p in enumerate(reqs):
        seen.setdefault(p.shape, i)
    for i in seen.values():
        submit(i)
    srv.drain()
    torch.cuda.synchronize()

    def run(arrivals):
        """arrivals[i] = seconds after start; returns per-request (latency, result)."""
        order = np.argsort(arrivals, kind="stable")
        ids, lat, res = {}, np.zeros(n_req), [None] * n_req
        k = 0
        start = time.perf_counter()
        while k < n_req or ids:
            now = time.perf_counter() - start
            while k < n_req and arrivals[order[k]] <= now:
                i = int(order[k])
                ids[i] = submit(i)
                k += 1
            q, r = srv.pending()
            if q == 0 and r == 0:
                if k < n_req:
                    time.sleep(max(0.0, arrivals[order[k]] - (time.perf_counter() - start)))
                continue
            if srv.step():
                t = time.perf_counter() - start
                for i in list(ids):
                    out = srv.result(ids[i])
                    if out is not None:
                        lat[i] = t - arrivals[i]
                        res[i] = out
                        del ids[i]
                        done = n_req - sum(r is None for r in res)
                        if done % 250 == 0:
                            print(f"serve: {done} of {n_req} retired", file=sys.stderr, flush=True)
        return lat, res, time.perf_counter() - start

    closed_lat, closed_res, makespan = run(np.zeros(n_req))
    sat = n_req / makespan

    def pct(x, q):
        return round(float(np.percentile(x, q)), 4) if len(x) else None

    # open loops: Poisson arrivals at each load factor x the closed-loop rate (the same
    # draws, scaled); the first factor's run is the reported one
    open_runs = []
    for load_factor in load_factors:
        rng = np.random.default_rng(seed)
        rate = load_factor * sat
        arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
        arr -= arr[0]
        lat_f, res_f, span_f = run(arr)
        ok_f = np.array([r.status[0] for r in res_f]) == hz.HZ_OK
        open_runs.append((load_factor, rate, lat_f, res_f, span_f, {
            "arrival_rate_per_s": round(rate, 3), "load_factor": load_factor, "span_s": round(span_f, 3),
            "solves_per_s": round(n_req / span_f, 3),
            "converged": int(ok_f.sum()), "not_converged": int((~ok_f).sum()),
            "p50_s": pct(lat_f[ok_f], 50), "p99_s": pct(lat_f[ok_f], 99),
            "p50_all_s": pct(lat_f, 50), "p99_all_s": pct(lat_f, 99)}))
    load_factor, rate, lat, res, span, open_rec = open_runs[0]
    status = np.array([r.status[0] for r in res])
    iters = np.array([r.iters[0] for r in res])
    vox = np.array([np.prod(p.shape) for p in reqs], dtype=np.float64)
    ok = status == hz.HZ_OK
    closed_ok = np.array([r.status[0] for r in closed_res]) == hz.HZ_OK

    # which requests reach 1e-6 within the budget, by microstructure kind and contrast
    # decade: the basic scheme's rate degrades like 1 - O(1/C) on percolating stiff phases
    resid = np.array([r.residual[0] for r in res])
    by_contrast = []
    for kind in ("spheres", "polycrystal"):
        for d in range(1, 6):
            sel = np.array([p.info["kind"] == kind and d <= np.log10(p.info["contrast"]) < d + 1 for p in reqs])
            if not sel.any():
                continue
            by_contrast.append({"kind": kind, "contrast": f"1e{d}..1e{d + 1}", "n": int(sel.sum()),
                                "converged": int(ok[sel].sum()),
                                "median_iters_converged": (int(np.median(iters[sel & ok])) if (sel & ok).any()
                                                           else None),
                                "median_residual_not_converged": (float(np.median(resid[sel & ~ok]))
                                                                  if (sel & ~ok).any() else None)})
    names = {hz.HZ_OK: "ok", hz.HZ_NOT_CONVERGED: "not_converged", hz.HZ_STAGNATED: "stagnated",
             hz._abi.HZ_EDIVERGED: "diverged"}
    return {
        "workload": f"{n_req} requests: n in {{32,48,64,96,128,160,192}}^3, Boolean spheres (R=n/16, vf 0.3) or "
                    f"200-grain cubic polycrystal (Zener ratio = contrast), contrast log-uniform 1e1..1e6, one unit "
                    f"load each, FP32+refine to 1e-6, max_iters {max_iters}",
        "latency_basis": "p50/p99 over the requests that reached 1e-6; the others (max_iters reached) are "
                         "counted beside them and enter only the *_all_s figures",
        "closed_loop": {"makespan_s": round(makespan, 3), "solves_per_s": round(sat, 3),
                        "converged": int(closed_ok.sum()), "not_converged": int((~closed_ok).sum()),
                        "p50_s": pct(closed_lat[closed_ok], 50), "p99_s": pct(closed_lat[closed_ok], 99),
                        "p50_all_s": pct(closed_lat, 50), "p99_all_s": pct(closed_lat, 99)},
        "open_loop": open_rec,
        **({"open_loop_other_loads": [o[5] for o in open_runs[1:]]} if len(open_runs) > 1 else {}),
        "status_counts": {names.get(int(c), str(int(c))): int((status == c).sum()) for c in np.unique(status)},
        "by_contrast": by_contrast,
        "fp64_fallbacks": int(sum(int(r.precision_used[0]) == hz.HZ_FP64 for r in res)),
        "mean_fp32_iters": round(float(iters.mean()), 1),
        "voxel_iters_per_s_closed_loop": float((vox * iters).sum() / makespan),
        "arena_gib": round(arena / 2 ** 30, 2), "generation_s": round(gen_s, 1), "streams": streams,
    }


def headline(a, hz, np, torch, p, g, copy_gbps):
    """The headline: exactly `steps` iterations of the six loads of the 128^3 workload
    in FP64, after `warmup` untimed ones; the dominant kernel's roofline from HIP events
    around its launches over the timed iterations."""
    N1, N2, N3 = p.shape
    N = N1 * N2 * N3
    S = (N1 // 2 + 1) * N2 * N3
    g.bind(hz.HZ_FP64, 6)
    torch.cuda.synchronize()
    schemes = {"auto": hz.HZ_SCHEME_AUTO, "spectral": hz.HZ_SCHEME_SPECTRAL, "stencil": hz.HZ_SCHEME_STENCIL}
    sch = schemes[a.scheme]
    # warmup, then exactly `steps` iterations of all six loads
    if a.warmup > 0:
        g.solve(p.loads, C0=p.C0, fixed_iters=a.warmup - 1, check_every=1 << 20, scheme=sch)
    # per-kernel breakdown (untimed): HIP events around every launch of a short run
    g.profile(True)
    g.solve(p.loads, C0=p.C0, fixed_iters=max(4, a.steps // 4) - 1, check_every=1 << 20, scheme=sch)
    torch.cuda.synchronize()
    g.profile(False)
    prof = g.profile_read()
    dom_name = max(prof, key=lambda k: prof[k][0])
    # the timed region carries HIP events around every launch of the dominant kernel on
    # the library's stream: its roofline comes from exactly the iterations timed
    torch.cuda.synchronize()
    g.profile(True, only=dom_name)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = g.solve(p.loads, C0=p.C0, fixed_iters=a.steps - 1, check_every=1 << 20, scheme=sch)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.profile(False)
    timed = g.profile_read()
    assert np.all(r.iters == a.steps - 1) and set(timed) == {dom_name}
    value = N * 6 * a.steps / dt
    log(f"bench: {a.steps} steps in {dt * 1e3:.1f} ms -> {value / 1e9:.3f} G voxel-iters/s")
    # the other realisation, same workload, for context (not the headline value)
    other = hz.HZ_SCHEME_SPECTRAL if any(k.startswith("stencil") for k in prof) else hz.HZ_SCHEME_STENCIL
    alt = None
    if g.scheme_available(other):
        k2 = max(4, a.steps // 4)
        g.solve(p.loads, C0=p.C0, fixed_iters=1, check_every=1 << 20, scheme=other)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.solve(p.loads, C0=p.C0, fixed_iters=k2 - 1, check_every=1 << 20, scheme=other)
        torch.cuda.synchronize()
        alt = {"scheme": "spectral" if other == hz.HZ_SCHEME_SPECTRAL else "stencil", "steps": k2,
               "voxel_iters_per_s": N * 6 * k2 / (time.perf_counter() - t1)}
        log(f"bench: other scheme {alt}")

    # roofline of the dominant kernel from the library's HIP events on its stream, over
    # the timed iterations
    kind, prec = dom_name.rsplit("_", 1)
    ms, cnt = timed[dom_name]
    per_launch_bytes = kernel_bytes(kind, S, N, 6, 16 if prec == "f64" else 8)
    avg_s = ms / cnt / 1e3
    achieved = per_launch_bytes / avg_s / 1e9
    # HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs of this
    # workload, while the sources are the ones they were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"iteration_boolean{N1}_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        k = t.get("kernels", {}).get(dom_name)
        if t.get("source_digest") == source_digest() and k and k.get("problems") == 6:
            traffic = k.get("bytes_per_launch")
    roof = {"bound": "hbm", "kernel": f"{kind}_{prec}", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_launch": per_launch_bytes,
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": cnt, "device_copy_GBps": round(copy_gbps, 1)}
    total = sum(v[0] for v in prof.values())
    per_kernel = kernel_rates(prof, S, N, 6)
    for k, v in per_kernel.items():
        v["share"] = round(prof[k][0] / total, 3)
    # whole-iteration fraction: algorithmic bytes of one iteration of the scheme used
    scheme = "stencil" if any(k.startswith("stencil") for k in prof) else "spectral"
    model_bytes = iteration_bytes(scheme, S, N, 16) / N
    iter_frac = value * model_bytes / (HBM_PEAK_GBS * 1e9)
    return {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Boolean spheres, random-free stiffness)",
        "config": {"workload": f"boolean{N1}_contrast1e3_6loads", "grid": [N1, N2, N3], "loads": 6,
                   "precision": "fp64", "vf": round(p.info["vf"], 4), "n_spheres": p.info["n_spheres"],
                   "parallelism": "single GPU"},
        "roofline": roof, "scheme": scheme, "other_scheme": alt, "bytes_per_voxel_iteration": round(model_bytes, 1),
        "iteration_roofline_frac": round(iter_frac, 4), "per_kernel": per_kernel,
    }


LEGS = ("iter", "ceff", "full", "ttt", "serve", "cpu", "sweep", "compare")
DEFAULT_LEGS = ("iter", "ceff", "full", "ttt", "compare", "serve", "cpu")
FULL = ("voronoi256", "spheres192x192x320")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--legs", default=",".join(DEFAULT_LEGS),
                    help="legs to run, of " + ",".join(LEGS) + " (the JSON line carries the headline value "
                         "only with 'iter')")
    ap.add_argument("--full", default=",".join(FULL), help="full-size workloads, of " + ",".join(FULL))
    ap.add_argument("--full-steps", type=int, default=24,
                    help="passes of the longer full-size run (the shorter one runs a sixth of them)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1e-6 comparison")
    ap.add_argument("--scheme", choices=["auto", "spectral", "stencil"], default="auto")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-n", type=int, default=200, help="requests in the serving stream")
    ap.add_argument("--serve-max-iters", type=int, default=1000, help="iteration budget per served request")
    ap.add_argument("--serve-streams", type=int, default=4, help="streams the server spreads its groups over")
    ap.add_argument("--serve-loads", default="0.7",
                    help="open-loop load factors (x the closed-loop rate), comma separated; the first is reported")
    ap.add_argument("--sweep-grids", default="256x256x256,192x192x320", help="grids of the contrast sweep")
    ap.add_argument("--sweep-contrasts", default="0,1e-4,1e-2,10,1e2,1e3,1e4,1e6,1e8",
                    help="inclusion-to-matrix stiffness ratios of the contrast sweep")
    ap.add_argument("--compare-parts", default="void,hard,contrast,rates",
                    help="parts of the compare leg: void (cubic void of Sec. 3.2), hard (hard sphere of "
                         "Sec. 3.3), contrast (iterates versus contrast, Sec. 3.4), rates (iteration rates)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on more than one GPU are not supported",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    legs = set(a.legs.split(",")) if a.legs else set()
    full = [w for w in a.full.split(",") if w] if a.full else []
    if legs - set(LEGS) or set(full) - set(FULL):
        ap.error("unknown leg or workload")
    legs -= {"cpu"} if a.no_cpu else set()
    legs -= {"ttt"} if a.no_ttt else set()
    legs -= {"serve"} if a.no_serve else set()

    import numpy as np
    import torch

    import hz_synth as syn
    import paper_2405_11168_amd as hz

    torch.cuda.set_device(0)
    if a.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    # context for the roofline: what a plain 1 GiB device-to-device copy reaches on this
    # GPU (read + write bytes over time), next to the published 8 TB/s
    x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    copy_gbps = 10 * 2 * (1 << 30) / (time.perf_counter() - t0) / 1e9
    del x, y
    log(f"bench: device copy {copy_gbps:.0f} GB/s")
    out = {}
    p = g = None
    if legs & {"iter", "ceff", "cpu"}:
        log(f"bench: building workload boolean{a.n} (contrast 1e3, 6 loads)")
        p = syn.boolean128(n=a.n)
        g = hz.Grid(*p.shape)
        g.set_material(p.C, p.phase)
    if "iter" in legs:
        out.update(headline(a, hz, np, torch, p, g, copy_gbps))
    if "ceff" in legs:
        log("bench: converged C_eff of the headline workload (FP64 and FP32+refine, eps < 1e-8)")
        out["ceff_converged"] = ceff_leg(hz, np, torch, p, g)
        log(f"bench: ceff {out['ceff_converged']}")
    poly = gp = None
    if "ttt" in legs or "voronoi256" in full and "full" in legs:
        log("bench: building the 256^3 Voronoi polycrystal")
        poly = syn.polycrystal()
        gp = hz.Grid(*poly.shape)
        gp.set_material(poly.C, poly.phase)
    if "full" in legs:
        out["full_size"] = {}
        for w in full:
            if w == "voronoi256":
                q, gq, name = poly, gp, "voronoi256_200grains_cubic_6loads"
            else:
                q = syn.sphere_contrast((192, 192, 320), 10.0)
                gq = hz.Grid(*q.shape)
                gq.set_material(q.C, q.phase)
                name = "spheres192x192x320_vf0.25_contrast10_6loads"
            loads = np.stack([syn.unit_load(J) for J in range(6)])
            out["full_size"][w] = full_size_leg(hz, np, torch, name, q, gq, loads, K1=max(2, a.full_steps // 6),
                                                K2=max(a.full_steps, 4))
            log(f"bench: full size {w}: {out['full_size'][w]}")
            if gq is not gp:
                del gq
    if "ttt" in legs:
        out["time_to_1e-6"] = time_to_tol(hz, np, torch, poly, gp)
        log(f"bench: ttt {out['time_to_1e-6']}")
    del gp
    if "sweep" in legs:
        grids = [tuple(int(v) for v in t.split("x")) for t in a.sweep_grids.split(",") if t]
        out["contrast_sweep"] = sweep_leg(syn, hz, np, torch, grids, [float(c) for c in a.sweep_contrasts.split(",")])
    if "compare" in legs:
        log("bench: comparison Green operators (cubic void of Sec. 3.2, iteration rates)")
        out["green_operators"] = compare_leg(syn, hz, np, torch, parts=tuple(a.compare_parts.split(",")))
    if "serve" in legs:
        log(f"bench: serving leg ({a.serve_n} requests)")
        out["serving"] = serving_leg(syn, hz, np, torch, a.serve_n, a.serve_max_iters, streams=a.serve_streams,
                                     load_factors=tuple(float(v) for v in a.serve_loads.split(",")))
        log(f"bench: serving {out['serving']}")
    if "cpu" in legs:
        log("bench: CPU oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(p)
        log(f"bench: cpu {out['cpu_baseline']}")
    if "iter" not in legs:
        out = {"legs": sorted(legs), **out}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

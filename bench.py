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
  cpu_baseline   the CPU oracle timed on the host on a bounded sample
  time_to_1e-6   FP32+refinement vs plain FP64 device time to an FP64-verified
                 residual of 1e-6 on the 256^3 Voronoi polycrystal (6 loads)
  serving        a seeded stream of solve requests (grid sizes 32..192^3, Boolean
                 spheres or cubic polycrystals, contrast log-uniform 1e1..1e6, one
                 load each, FP32+refine to 1e-6) through the solve server: closed-loop
                 saturation throughput, then Poisson arrivals at 0.7x that rate with
                 p50/p99 latency from arrival to result
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


def cpu_baseline(problem, max_seconds=15.0):
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
    return {"value": n * iters / dt, "unit": "voxel-iters/s", "cores": tetra.WORKERS, "kind": "oracle",
            "sample": f"1 of 6 loads, {iters} iteration(s) of the 128^3 workload (FP64 numpy+scipy.fft), "
                      f"{dt:.1f} s wall"}


def time_to_tol(syn, hz, np, torch, n):
    """Device time to an FP64-verified residual of 1e-6 on the periodic Voronoi
    polycrystal (200 cubic grains C11=168, C12=121, C44=75, random orientations,
    6 unit loads): plain FP64 iterations against FP32 iterations anchored by FP64
    sweeps.  Each variant runs three times: a warmup, a run with HIP events around
    every launch (per-kernel times), and the reported run without them."""
    p = syn.polycrystal(shape=(n, n, n))
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
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
        out[name] = {"seconds_to_1e-6": round(float(np.max(r.seconds_to_1e6)), 4), "wall_s": round(wall, 4),
                     "iters": int(np.max(r.iters)), "outer_rounds": int(np.max(r.outer_rounds)),
                     "residual": float(np.max(r.residual)),
                     "kernel_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in prof.items()}}
    out["speedup"] = round(out["fp64"]["seconds_to_1e-6"] / out["fp32_refine"]["seconds_to_1e-6"], 3)
    m64, m32 = res["fp64"].mean_sigma, res["fp32_refine"].mean_sigma
    out["ceff_rel_diff_fp32r_vs_fp64"] = float(np.abs(m32 - m64).max() / np.abs(m64).max())
    del g
    return out


def serving_leg(syn, hz, np, torch, n_req, max_iters, load_factor=0.7, seed=5):
    """Closed loop (all requests at t=0) for the saturation rate, then an open
    loop with Poisson arrivals at load_factor x that rate.  Latency = result
    ready (the server step that retired the request) - arrival time."""
    t0 = time.perf_counter()
    reqs = [syn.serving_request(i) for i in range(n_req)]
    grids = []
    for p in reqs:
        g = hz.Grid(*p.shape)
        g.set_material(p.C, p.phase)
        grids.append(g)
    gen_s = time.perf_counter() - t0
    need = [hz.request_bytes(g, hz.HZ_FP32_REFINE, 1) for g in grids]
    arena = min(int(1.05 * sum(need)), 160 << 30)
    srv = hz.Server(arena, max_problems=n_req + 8, check_every=8)

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
        return lat, res, time.perf_counter() - start

    closed_lat, closed_res, makespan = run(np.zeros(n_req))
    sat = n_req / makespan
    rng = np.random.default_rng(seed)
    rate = load_factor * sat
    arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
    arr -= arr[0]
    lat, res, span = run(arr)
    status = np.array([r.status[0] for r in res])
    iters = np.array([r.iters[0] for r in res])
    vox = np.array([np.prod(p.shape) for p in reqs], dtype=np.float64)
    ok = status == hz.HZ_OK
    names = {hz.HZ_OK: "ok", hz.HZ_NOT_CONVERGED: "not_converged", hz.HZ_STAGNATED: "stagnated",
             hz._abi.HZ_EDIVERGED: "diverged"}
    return {
        "workload": f"{n_req} requests: n in {{32,48,64,96,128,160,192}}^3, Boolean spheres (R=n/16, vf 0.3) or "
                    f"200-grain cubic polycrystal (Zener ratio = contrast), contrast log-uniform 1e1..1e6, one unit "
                    f"load each, FP32+refine to 1e-6, max_iters {max_iters}",
        "closed_loop": {"makespan_s": round(makespan, 3), "solves_per_s": round(sat, 3),
                        "p50_s": round(float(np.percentile(closed_lat, 50)), 4),
                        "p99_s": round(float(np.percentile(closed_lat, 99)), 4)},
        "open_loop": {"arrival_rate_per_s": round(rate, 3), "load_factor": load_factor, "span_s": round(span, 3),
                      "solves_per_s": round(n_req / span, 3),
                      "p50_s": round(float(np.percentile(lat, 50)), 4),
                      "p99_s": round(float(np.percentile(lat, 99)), 4),
                      "p50_converged_s": round(float(np.percentile(lat[ok], 50)), 4) if ok.any() else None,
                      "p99_converged_s": round(float(np.percentile(lat[ok], 99)), 4) if ok.any() else None},
        "status_counts": {names.get(int(c), str(int(c))): int((status == c).sum()) for c in np.unique(status)},
        "fp64_fallbacks": int(sum(int(r.precision_used[0]) == hz.HZ_FP64 for r in res)),
        "mean_fp32_iters": round(float(iters.mean()), 1),
        "voxel_iters_per_s_closed_loop": float((vox * iters).sum() / makespan),
        "arena_gib": round(arena / 2 ** 30, 2), "generation_s": round(gen_s, 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1e-6 comparison")
    ap.add_argument("--ttt-n", type=int, default=256, help="grid size of the time-to-1e-6 polycrystal")
    ap.add_argument("--scheme", choices=["auto", "spectral", "stencil"], default="auto")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-n", type=int, default=64, help="requests in the serving stream")
    ap.add_argument("--serve-max-iters", type=int, default=1000, help="iteration budget per served request")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on more than one GPU are not supported",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

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
    log(f"bench: building workload boolean{a.n} (contrast 1e3, 6 loads)")
    p = syn.boolean128(n=a.n)
    N1, N2, N3 = p.shape
    N = N1 * N2 * N3
    S = (N1 // 2 + 1) * N2 * N3
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
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
    kinds = {}
    for name, (ms, cnt) in prof.items():
        kind, prec = name.rsplit("_", 1)
        kinds[name] = (kind, prec, ms, cnt)
    kind, prec = dom_name.rsplit("_", 1)
    ms, cnt = timed[dom_name]
    per_launch_bytes = kernel_bytes(kind, S, N, 6, 16 if prec == "f64" else 8)
    avg_s = ms / cnt / 1e3
    achieved = per_launch_bytes / avg_s / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{kind}_{prec}_boolean128_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        if t.get("source_digest") == source_digest():
            traffic = t.get("bytes_per_launch")
    roof = {"bound": "hbm", "kernel": f"{kind}_{prec}", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_launch": per_launch_bytes,
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": cnt, "device_copy_GBps": round(copy_gbps, 1)}
    per_kernel = {k: {"ms_per_launch": round(v[2] / v[3], 4), "share": round(v[2] / sum(x[2] for x in kinds.values()), 3)}
                  for k, v in kinds.items()}
    # whole-iteration fraction: algorithmic bytes of one iteration of the scheme used
    scheme = "stencil" if any(k.startswith("stencil") for k in prof) else "spectral"
    model_bytes = iteration_bytes(scheme, S, N, 16) / N
    iter_frac = value * model_bytes / (HBM_PEAK_GBS * 1e9)

    ttt = None
    if not a.no_ttt:
        ttt = time_to_tol(syn, hz, np, torch, a.ttt_n)
        log(f"bench: ttt {ttt}")

    serving = None
    if not a.no_serve:
        log(f"bench: serving leg ({a.serve_n} requests)")
        serving = serving_leg(syn, hz, np, torch, a.serve_n, a.serve_max_iters)
        log(f"bench: serving {serving}")

    cpu = None
    if not a.no_cpu:
        log("bench: CPU oracle baseline (bounded sample)")
        cpu = cpu_baseline(p)
        log(f"bench: cpu {cpu}")

    out = {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Boolean spheres, random-free stiffness)",
        "config": {"workload": f"boolean{N1}_contrast1e3_6loads", "grid": [N1, N2, N3], "loads": 6,
                   "precision": "fp64", "vf": round(p.info["vf"], 4), "n_spheres": p.info["n_spheres"],
                   "parallelism": "single GPU"},
        "roofline": roof, "scheme": scheme, "other_scheme": alt, "bytes_per_voxel_iteration": round(model_bytes, 1),
        "iteration_roofline_frac": round(iter_frac, 4),
        "per_kernel": per_kernel, "cpu_baseline": cpu, "time_to_1e-6": ttt, "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

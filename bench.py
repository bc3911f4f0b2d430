#!/usr/bin/env python3
"""Benchmark of the tetrahedral-stencil basic scheme on one MI355X.

Workload (the headline configuration): 128^3 periodic cell, Boolean model of
overlapping spheres (radius 8, seeded, 30% volume fraction), stiffness
contrast 1e3 (nu = 0.3), all six unit macroscopic strains solved as one batch
in FP64 (the effective-stiffness computation).  A "step" is one iteration of
Algorithm 1 over all six loads: expand, six 1D FFT passes, constitutive law,
Green-operator update and FP64 residual reduction.

Prints ONE JSON line:
  value          voxel-iterations/s (128^3 voxels x 6 loads x steps / timed seconds)
  roofline       the dominant kernel's algorithmic bytes per launch / its mean
                 HIP-event duration, against 8 TB/s
  cpu_baseline   the CPU oracle timed on the host on a bounded sample
  time_to_1e-6   FP32+refinement vs plain FP64 device time to an FP64-verified
                 residual of 1e-6 on the 256^3 Voronoi polycrystal (6 loads)
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
    for f in ("hz_kernels.hip", "hz_fft.h", "hz_internal.h", "hz_api.cpp"):
        with open(os.path.join(ROOT, "paper_2405_11168_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bytes(kind, S, N, nloads, csz):
    """Algorithmic HBM bytes of one launch of a pass over `nloads` problems:
    complex spectra moved (S complex elements per component, csz bytes each)."""
    units = {
        "zexpand": 3 + 12,         # read u (3), write 12 strain spectra
        "yinv": 24, "yfwd": 24,    # read 12, write 12
        "xpass": 24,               # read 12, write 12 (+ phase map)
        "zcontract": 12 + 3 + 3,   # read 12 stress spectra + u, write u
    }
    if kind not in units:
        return None
    b = units[kind] * S * csz
    if kind == "xpass":
        b += 2 * N
    return b * nloads


def cpu_baseline(problem, max_seconds=25.0):
    """The oracle (FP64 numpy/scipy, Algorithm 1) on a bounded sample: one load,
    a few iterations of the same 128^3 workload, timed on the host."""
    from oracle import tetra

    n = problem.phase.size
    iters = 1
    t0 = time.perf_counter()
    tetra.basic_scheme(problem.phase, problem.C, problem.C0, problem.loads[0], fixed_iters=iters - 1,
                       keep_fields=False)
    dt = time.perf_counter() - t0
    k = max(1, min(4, int(max_seconds / max(dt, 1e-3))))
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
    sweeps.  Each variant runs twice; the second run is reported."""
    p = syn.polycrystal(shape=(n, n, n))
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    out = {"workload": f"voronoi{n}_200grains_cubic_6loads", "tol": 1e-6}
    res = {}
    for prec, name in ((hz.HZ_FP64, "fp64"), (hz.HZ_FP32_REFINE, "fp32_refine")):
        g.bind(prec, 6)
        for rep in range(2):
            if rep == 1:
                g.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.solve(p.loads, C0=p.C0, tol=1e-6, precision=prec, check_every=4)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        g.profile(False)
        prof = g.profile_read()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1e-6 comparison")
    ap.add_argument("--ttt-n", type=int, default=256, help="grid size of the time-to-1e-6 polycrystal")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU: multi-GPU runs are not part of it",
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
    log(f"bench: building workload boolean{a.n} (contrast 1e3, 6 loads)")
    p = syn.boolean128(n=a.n)
    N1, N2, N3 = p.shape
    N = N1 * N2 * N3
    S = (N1 // 2 + 1) * N2 * N3
    g = hz.Grid(*p.shape)
    g.set_material(p.C, p.phase)
    g.bind(hz.HZ_FP64, 6)
    torch.cuda.synchronize()

    # warmup, then exactly `steps` iterations of all six loads
    if a.warmup > 0:
        g.solve(p.loads, C0=p.C0, fixed_iters=a.warmup - 1, check_every=1 << 20)
    torch.cuda.synchronize()
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = g.solve(p.loads, C0=p.C0, fixed_iters=a.steps - 1, check_every=1 << 20)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.profile(False)
    prof = g.profile_read()
    assert np.all(r.iters == a.steps - 1)
    value = N * 6 * a.steps / dt
    log(f"bench: {a.steps} steps in {dt * 1e3:.1f} ms -> {value / 1e9:.3f} G voxel-iters/s")

    # roofline of the dominant kernel from the library's HIP events on its stream
    kinds = {}
    for name, (ms, cnt) in prof.items():
        kind, prec = name.rsplit("_", 1)
        kinds[name] = (kind, prec, ms, cnt)
    dom = max(kinds.values(), key=lambda t: t[2])
    kind, prec, ms, cnt = dom
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
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": cnt}
    per_kernel = {k: {"ms_per_launch": round(v[2] / v[3], 4), "share": round(v[2] / sum(x[2] for x in kinds.values()), 3)}
                  for k, v in kinds.items()}
    # whole-iteration fraction against the 105-unit byte model of one iteration
    model_bytes = (105 * S * 16 + 2 * N) / N
    iter_frac = value * model_bytes / (HBM_PEAK_GBS * 1e9)

    ttt = None
    if not a.no_ttt:
        ttt = time_to_tol(syn, hz, np, torch, a.ttt_n)
        log(f"bench: ttt {ttt}")

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
        "roofline": roof, "iteration_roofline_frac_105unit_model": round(iter_frac, 4),
        "per_kernel": per_kernel, "cpu_baseline": cpu, "time_to_1e-6": ttt, "serving": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

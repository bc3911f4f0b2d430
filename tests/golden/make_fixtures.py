"""Write the converged-oracle fixtures of the full-size workloads (CPU only).

Every stored number comes from the FP64 oracle (``oracle.tetra.basic_scheme``,
Algorithm 1 with the stop rule of eqs. L2-norm and tolerance) run on inputs
from the seeded generators of ``hz_synth``; nothing here touches the HIP
library.  Each fixture keeps, for one load of one workload:

* ``history``        eps_k of every iterate k = 0 .. iters (eq. tolerance);
* ``mean_history``   <sigma>_k of every iterate (tensor comps 11,22,33,23,13,12);
* ``iters``          the first k with eps_k < tol_run (the run stops there);
* ``mean_sigma``     <sigma> of that iterate: the converged column of C_eff
                     (eq. final_fields) used as the reference of inexact solves.

The GPU tests read the iterate at which an FP64 solve stopped out of
``mean_history`` (iterate-matched parity) and compare an FP32+refine solve with
``mean_sigma``.  ``serving_stream_requests`` keeps the same quantities for ten small
requests of the serving stream itself.  At 256^3 one oracle iteration takes tens of
seconds on 8 cores, so the whole set takes about two hours; run it once:

    python tests/golden/make_fixtures.py [name ...]
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hz_synth as syn  # noqa: E402
from oracle import tetra  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_RUN = 1e-9
CITATION = ("Algorithm 1 (Sec. 2.6): u(q) = 0, update of eq. basic_scheme_dep_2 with Omega of eq. "
            "Green_tensor; eps_k of eqs. L2-norm and tolerance; <sigma> = (<sigma^T1> + <sigma^T2>)/2 "
            "of eq. final_fields")


def _cases():
    """name -> (problem builder, recipe text, load index)."""
    return {
        "voronoi256_load0": (lambda: syn.polycrystal(), "hz_synth.polycrystal() (256^3, 200 grains, seed 3)", 0),
        "voronoi256_load3": (lambda: syn.polycrystal(), "hz_synth.polycrystal() (256^3, 200 grains, seed 3)", 3),
        "spheres256_c10": (lambda: syn.sphere_contrast((256, 256, 256), 10.0),
                           "hz_synth.sphere_contrast((256, 256, 256), 10.0) (R 8, vf 0.25, seed 4)", 0),
        "spheres192x192x320_c10": (lambda: syn.sphere_contrast((192, 192, 320), 10.0),
                                   "hz_synth.sphere_contrast((192, 192, 320), 10.0) (R 8, vf 0.25, seed 4)", 0),
    }


STREAM_PICKS = 10


def stream_picks():
    """Indices of the first STREAM_PICKS requests of the serving stream with n <= 48 and
    contrast < 10^1.5: small, moderate-contrast requests the oracle converges in seconds."""
    out, i = [], 0
    while len(out) < STREAM_PICKS:
        n, kind, contrast, J = syn.serving_request_params(i)
        if n <= 48 and contrast < 10 ** 1.5:
            out.append(i)
        i += 1
    return out


def make_stream(name="serving_stream_requests"):
    """Converged oracle runs of requests of the serving stream itself (hz_synth.serving_request)."""
    reqs = []
    t0 = time.time()
    for i in stream_picks():
        p = syn.serving_request(i)
        ref = tetra.basic_scheme(p.phase, p.C, p.C0, p.loads[0], tol=TOL_RUN, max_iters=2000, keep_fields=False)
        assert ref.converged, (i, ref.residual)
        reqs.append({"index": i, "shape": list(p.shape), "kind": p.info["kind"], "contrast": p.info["contrast"],
                     "load": p.loads[0].tolist(), "iters": int(ref.iters), "history": ref.history.tolist(),
                     "mean_history": ref.mean_history.tolist(), "mean_sigma": ref.mean_sigma.tolist()})
        print(f"  request {i}: {p.shape[0]}^3 {p.info['kind']} contrast {p.info['contrast']:.1f}, "
              f"{ref.iters} iterations", flush=True)
    out = {
        "name": name,
        "citation": CITATION,
        "recipe": "hz_synth.serving_request(i) for the first %d requests with n <= 48 and contrast < 10^1.5"
                  % STREAM_PICKS,
        "tol_run": TOL_RUN,
        "requests": reqs,
        "oracle_wall_s": round(time.time() - t0, 1),
        "host": f"{platform.processor() or platform.machine()}, {os.cpu_count()} cpus, numpy {np.__version__}",
        "command": "python tests/golden/make_fixtures.py " + name,
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {len(reqs)} requests -> {path}", flush=True)


def make(name):
    if name == "serving_stream_requests":
        return make_stream(name)
    build, recipe, J = _cases()[name]
    p = build()
    E = p.loads[J]
    t0 = time.time()
    ref = tetra.basic_scheme(p.phase, p.C, p.C0, E, tol=TOL_RUN, max_iters=600, keep_fields=False)
    wall = time.time() - t0
    assert ref.converged, (name, ref.residual)
    out = {
        "name": name,
        "citation": CITATION,
        "recipe": recipe,
        "shape": list(p.shape),
        "load_index": J,
        "load": E.tolist(),
        "C0": p.C0.tolist(),
        "tol_run": TOL_RUN,
        "iters": int(ref.iters),
        "history": ref.history.tolist(),
        "mean_history": ref.mean_history.tolist(),
        "mean_sigma": ref.mean_sigma.tolist(),
        "oracle_wall_s": round(wall, 1),
        "host": f"{platform.processor() or platform.machine()}, {os.cpu_count()} cpus, numpy {np.__version__}",
        "command": "python tests/golden/make_fixtures.py " + name,
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {ref.iters} iterations to {TOL_RUN:g} in {wall:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(_cases()) + ["serving_stream_requests"]
    for n in names:
        make(n)

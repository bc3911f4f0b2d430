"""MI355X (gfx950) solver for the tetrahedral-stencil FFT homogenization method
(Finel, arXiv 2405.11168): the displacement-based basic scheme of Algorithm 1
iterated entirely in hand-written HIP kernels behind the C ABI of include/hz.h.

PyTorch provides device memory (the caller-owned workspace) and the HIP
stream; every step of the iteration runs in libhz.so.  There is no CPU path:
without the built library the solver raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (HZ_EDIVERGED, HZ_FP32_REFINE, HZ_FP64, HZ_LOAD_STRAIN, HZ_LOAD_STRESS, HZ_NOT_CONVERGED, HZ_OK,
                   HZ_PENDING, HZ_SCHEME_AUTO, HZ_SCHEME_SPECTRAL, HZ_SCHEME_STENCIL, HZ_SCHEME_STRAIN,
                   HZ_GREEN_TETRA, HZ_GREEN_ROTATED, HZ_GREEN_CONTINUOUS,
                   HZ_STAGNATED, HzError, check, hz_info, hz_opts)

__all__ = ["Grid", "Server", "SolveResult", "HZ_GREEN_TETRA", "HZ_GREEN_ROTATED", "HZ_GREEN_CONTINUOUS", "HZ_FP64", "HZ_FP32_REFINE", "HZ_LOAD_STRAIN", "HZ_LOAD_STRESS", "HzError",
           "reference_medium", "lib"]


def lib():
    return _abi.load()


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def reference_medium(C):
    """Reference medium of the library's automatic rule for phases C[P,6,6] (host only)."""
    C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, 6, 6)
    out = np.zeros(36)
    check(lib().hz_reference_medium(len(C), _dptr(C), _dptr(out)))
    return out.reshape(6, 6)


def _opts(tol=1e-8, max_iters=2000, precision=HZ_FP64, C0=None, fixed_iters=-1, check_every=8, inner_rho=1e-3,
          inner_max=400, scheme=HZ_SCHEME_AUTO, loading=HZ_LOAD_STRAIN):
    o = hz_opts()
    lib().hz_default_opts(ctypes.byref(o))
    o.tol = tol
    o.max_iters = max_iters
    o.precision = precision
    o.fixed_iters = fixed_iters
    o.check_every = check_every
    o.inner_rho = inner_rho
    o.inner_max = inner_max
    o.scheme = scheme
    o.loading = loading
    if C0 is not None:
        o.ref_mode = 1
        o.ref_C[:] = np.asarray(C0, dtype=np.float64).reshape(36).tolist()
    return o


def _outcome(rc):
    """A solve's worst per-load status: a diverged load is an outcome (its info and
    outputs are written), every other negative code an error."""
    return rc if rc == HZ_EDIVERGED else check(rc)


def _result(sm, infos, rc, **kw):
    return SolveResult(
        mean_sigma=sm,
        status=np.array([i.status for i in infos]),
        iters=np.array([i.iters for i in infos]),
        outer_rounds=np.array([i.outer_rounds for i in infos]),
        residual=np.array([i.residual for i in infos]),
        seconds=np.array([i.seconds for i in infos]),
        seconds_to_1e6=np.array([i.seconds_to_1e6 for i in infos]),
        rc=rc, wall_seconds=np.array([i.wall_seconds for i in infos]),
        Ebar=np.array([list(i.Ebar) for i in infos]),
        precision_used=np.array([i.precision_used for i in infos]), **kw)


@dataclass
class SolveResult:
    mean_sigma: np.ndarray          # [n_loads, 6] tensor comps
    status: np.ndarray              # [n_loads]
    iters: np.ndarray
    outer_rounds: np.ndarray
    residual: np.ndarray
    seconds: np.ndarray
    seconds_to_1e6: np.ndarray
    rc: int
    wall_seconds: np.ndarray | None = None
    Ebar: np.ndarray | None = None             # [n_loads, 6] mean strain of the reported iterate
    precision_used: np.ndarray | None = None   # [n_loads] HZ_FP64 also for a refinement that fell back
    trace_residual: np.ndarray | None = None   # [n_loads, T]
    trace_mean: np.ndarray | None = None       # [n_loads, T, 6]
    eps: np.ndarray | None = None              # [n_loads, 6, N3, N2, N1]
    sigma: np.ndarray | None = None


class Grid:
    """One periodic N1 x N2 x N3 cell (hz_grid handle) with a torch-owned workspace."""

    def __init__(self, n1: int, n2: int, n3: int):
        L = lib()
        h = ctypes.c_void_p()
        check(L.hz_create_grid(n1, n2, n3, ctypes.byref(h)))
        self._h = h
        self.shape = (n1, n2, n3)
        self._ws = None
        self._bound = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().hz_destroy_grid(h)
            except Exception:
                pass
            self._h = None

    # -- material ---------------------------------------------------------------
    def set_material(self, C, phase):
        """C: [P,6,6] Voigt stiffness; phase: [N3,N2,N1] ids (uint16)."""
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, 6, 6)
        phase = np.ascontiguousarray(phase, dtype=np.uint16)
        n1, n2, n3 = self.shape
        if phase.shape != (n3, n2, n1):
            raise ValueError(f"phase map must be [N3,N2,N1] = {(n3, n2, n1)}, got {phase.shape}")
        check(lib().hz_set_material(self._h, len(C), _dptr(C),
                                    phase.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))))
        self._bound = None

    def set_eigenstrain(self, eps0):
        """eps0: [P,6] per-phase eigenstrain (tensor comps), or None to clear."""
        if eps0 is None:
            check(lib().hz_set_eigenstrain(self._h, 0, None))
        else:
            e = np.ascontiguousarray(eps0, dtype=np.float64).reshape(-1, 6)
            check(lib().hz_set_eigenstrain(self._h, len(e), _dptr(e)))
        self._bound = None

    # -- workspace -------------------------------------------------------------
    def workspace_bytes(self, precision=HZ_FP64, n_loads=1) -> int:
        return check(lib().hz_workspace_bytes(self._h, precision, n_loads))

    def bind(self, precision=HZ_FP64, n_loads=1, device="cuda", stream=None):
        """Allocate the device workspace with torch and hand it to the library."""
        import torch

        nbytes = self.workspace_bytes(precision, n_loads)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        s = stream if stream is not None else torch.cuda.current_stream(self._ws.device)
        self._stream = s
        check(lib().hz_bind_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                      ctypes.c_void_p(s.cuda_stream), precision, n_loads))
        self._bound = (precision, n_loads)

    def _ensure(self, precision, n_loads):
        """Bind a workspace for at least n_loads loads (the strain-based scheme asks for 2 n)."""
        b = self._bound
        if b is None or b[0] != precision or b[1] < n_loads:
            self.bind(precision, n_loads)

    # -- solve -----------------------------------------------------------------
    def _prepare(self, nl, tol, max_iters, precision, C0, fixed_iters, trace, check_every, inner_rho, inner_max,
                 scheme, loading, u_init, Ebar_init, green=HZ_GREEN_TETRA):
        """Options struct and the host arrays it points to (kept alive by the caller)."""
        self._ensure(precision, 2 * nl if scheme == HZ_SCHEME_STRAIN else nl)
        o = _opts(tol, max_iters, precision, C0, fixed_iters, check_every, inner_rho, inner_max, scheme, loading)
        o.green = green
        T = (fixed_iters if fixed_iters >= 0 else max_iters) + 1
        keep = {}
        if trace:
            keep["tr"] = np.full((nl, T), np.nan)
            keep["tm"] = np.full((nl, T, 6), np.nan)
            o.trace_residual = _dptr(keep["tr"])
            o.trace_mean = _dptr(keep["tm"])
        if u_init is not None:
            n1, n2, n3 = self.shape
            u = np.asarray(u_init, dtype=np.complex128).reshape(nl, 3, n1 // 2 + 1, n3, n2)
            keep["ui"] = np.ascontiguousarray(np.stack([u.real, u.imag], axis=-1))
            o.u_init = _dptr(keep["ui"])
        if Ebar_init is not None:
            keep["eb"] = np.ascontiguousarray(np.asarray(Ebar_init, dtype=np.float64).reshape(nl, 6))
            o.Ebar_init = _dptr(keep["eb"])
        return o, keep

    def solve(self, E, tol=1e-8, max_iters=2000, precision=HZ_FP64, C0=None, fixed_iters=-1,
              fields=False, trace=False, check_every=8, inner_rho=1e-3, inner_max=400,
              scheme=HZ_SCHEME_AUTO, loading=HZ_LOAD_STRAIN, u_init=None, Ebar_init=None,
              fields_on_device=False, green=HZ_GREEN_TETRA) -> SolveResult:
        """E: [n_loads, 6] applied mean strains, or applied stresses with loading=HZ_LOAD_STRESS.
        u_init: optional [n_loads, 3, N1/2+1, N3, N2] complex displacement of iterate 0 (as
        returned by displacement()); Ebar_init: optional [n_loads, 6] mean strain of iterate 0
        under applied stress.  Together they resume a solve from a checkpoint.
        green: HZ_GREEN_TETRA (the paper's scheme) or a comparison operator,
        HZ_GREEN_ROTATED / HZ_GREEN_CONTINUOUS (FP64, spectral scheme).
        fields=True returns eps, sigma [n_loads, 6, N3, N2, N1] as numpy arrays, or with
        fields_on_device=True as float64 torch tensors on the workspace's device, written
        there by the library (no host round trip)."""
        E = np.ascontiguousarray(np.atleast_2d(np.asarray(E, dtype=np.float64)))
        nl = E.shape[0]
        o, keep = self._prepare(nl, tol, max_iters, precision, C0, fixed_iters, trace, check_every, inner_rho,
                                inner_max, scheme, loading, u_init, Ebar_init, green)
        sm = np.zeros((nl, 6))
        infos = (hz_info * nl)()
        n1, n2, n3 = self.shape
        eps = sig = None
        pe = ps = None
        if fields and fields_on_device:
            import torch

            eps = torch.empty((nl, 6, n3, n2, n1), dtype=torch.float64, device=self._ws.device)
            sig = torch.empty_like(eps)
            o.fields_on_device = 1
            pe = ctypes.cast(ctypes.c_void_p(eps.data_ptr()), ctypes.POINTER(ctypes.c_double))
            ps = ctypes.cast(ctypes.c_void_p(sig.data_ptr()), ctypes.POINTER(ctypes.c_double))
        elif fields:
            eps = np.zeros((nl, 6, n3, n2, n1))
            sig = np.zeros((nl, 6, n3, n2, n1))
            pe, ps = _dptr(eps), _dptr(sig)
        rc = _outcome(lib().hz_solve(self._h, nl, _dptr(E), ctypes.byref(o), _dptr(sm), pe, ps, infos))
        return _result(sm, infos, rc, trace_residual=keep.get("tr"), trace_mean=keep.get("tm"), eps=eps, sigma=sig)

    def effective_stiffness(self, tol=1e-8, max_iters=2000, precision=HZ_FP64, C0=None, fixed_iters=-1,
                            trace=False, check_every=8, inner_rho=1e-3, inner_max=400, scheme=HZ_SCHEME_AUTO,
                            green=HZ_GREEN_TETRA):
        """C_eff (6x6 Voigt) by hz_effective_stiffness: column J = <sigma> of the unit load
        gamma_J = 1, the six loads solved as one batch.  Returns (C_eff, SolveResult of the
        six loads in the order J = 0..5)."""
        o, keep = self._prepare(6, tol, max_iters, precision, C0, fixed_iters, trace, check_every, inner_rho,
                                inner_max, scheme, HZ_LOAD_STRAIN, None, None, green)
        Ce = np.zeros(36)
        infos = (hz_info * 6)()
        rc = _outcome(lib().hz_effective_stiffness(self._h, ctypes.byref(o), _dptr(Ce), infos))
        Ce = Ce.reshape(6, 6)
        return Ce, _result(Ce.T.copy(), infos, rc, trace_residual=keep.get("tr"), trace_mean=keep.get("tm"))

    def scheme_available(self, scheme) -> bool:
        return bool(check(lib().hz_scheme_available(self._h, scheme)))

    def displacement(self, load=0):
        """u~(q) of the reported iterate: complex [3, N1/2+1, N3, N2] (library phase convention)."""
        n1, n2, n3 = self.shape
        out = np.zeros((3, n1 // 2 + 1, n3, n2, 2))
        check(lib().hz_get_displacement(self._h, load, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    # -- profiling ---------------------------------------------------------------
    def profile(self, enable=True, only=None):
        """Start (enable) or stop per-kernel event timing; `only` names one entry of
        profile_read (e.g. "stencil_f64") to time that kernel's launches alone."""
        mode = 1 if enable else 0
        if enable and only is not None:
            n = 64
            names = (ctypes.c_char_p * n)()
            k = check(lib().hz_profile_read(self._h, n, names, None, None))
            idx = [names[i].decode() for i in range(min(k, n))]
            if only not in idx:
                raise ValueError(f"unknown kernel entry {only!r}")
            mode = 2 + idx.index(only)
        check(lib().hz_profile(self._h, mode))

    def profile_read(self):
        n = 64
        names = (ctypes.c_char_p * n)()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        k = check(lib().hz_profile_read(self._h, n, names, ms, cnt))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(k, n)) if cnt[i] > 0}


def request_bytes(grid: "Grid", precision=HZ_FP64, n_loads=1) -> int:
    """Arena bytes one served request on `grid` needs (buffers + shape and material tables)."""
    return check(lib().hz_request_bytes(grid._h, precision, n_loads))


class Server:
    """Solve server (hz_server handle): continuous batching of requests on a
    torch-owned workspace.  submit() queues a request, step() runs one tick
    (admission, check_every iterations of every active load, retirement),
    result() returns a finished request's SolveResult or None.  streams > 1 spreads the
    iterate groups of a tick over that many streams (hz_server_set_streams)."""

    def __init__(self, arena_bytes: int, max_problems=64, check_every=8, device="cuda", stream=None, streams=1):
        import torch

        fixed = check(lib().hz_server_bytes(max_problems))
        self._ws = torch.empty(fixed + int(arena_bytes), dtype=torch.uint8, device=device)
        s = stream if stream is not None else torch.cuda.current_stream(self._ws.device)
        self._stream = s
        h = ctypes.c_void_p()
        check(lib().hz_server_create(ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                     ctypes.c_void_p(s.cuda_stream), max_problems, check_every, ctypes.byref(h)))
        self._h = h
        self._nloads = {}
        if streams != 1:
            check(lib().hz_server_set_streams(h, streams))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().hz_server_destroy(h)
            except Exception:
                pass
            self._h = None

    def submit(self, grid: "Grid", E, tol=1e-8, max_iters=2000, precision=HZ_FP64, C0=None, inner_rho=1e-3,
               inner_max=400, scheme=HZ_SCHEME_AUTO, loading=HZ_LOAD_STRAIN) -> int:
        E = np.ascontiguousarray(np.atleast_2d(np.asarray(E, dtype=np.float64)))
        o = _opts(tol, max_iters, precision, C0, -1, 8, inner_rho, inner_max, scheme, loading)
        rid = ctypes.c_int64()
        check(lib().hz_server_submit(self._h, grid._h, E.shape[0], _dptr(E), ctypes.byref(o), ctypes.byref(rid)))
        self._nloads[rid.value] = E.shape[0]
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int32()
        check(lib().hz_server_step(self._h, ctypes.byref(n)))
        return n.value

    def pending(self):
        q = ctypes.c_int32()
        r = ctypes.c_int32()
        check(lib().hz_server_pending(self._h, ctypes.byref(q), ctypes.byref(r)))
        return q.value, r.value

    def result(self, rid: int, release=True):
        nl = self._nloads[rid]
        sm = np.zeros((nl, 6))
        infos = (hz_info * nl)()
        rc = _outcome(lib().hz_server_query(self._h, rid, _dptr(sm), infos))
        if rc == HZ_PENDING:
            return None
        if release:
            check(lib().hz_server_release(self._h, rid))
            del self._nloads[rid]
        return _result(sm, infos, rc)

    def drain(self, max_ticks=1 << 20):
        """Step until nothing is queued or running."""
        for _ in range(max_ticks):
            q, r = self.pending()
            if q == 0 and r == 0:
                return
            self.step()
        raise RuntimeError("server did not drain")

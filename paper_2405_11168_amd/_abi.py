"""ctypes declarations of the C ABI in include/hz.h (argument marshalling only)."""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint16, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhz.so")

HZ_OK = 0
HZ_NOT_CONVERGED = 1
HZ_STAGNATED = 2
HZ_PENDING = 3
HZ_EINVAL = -1
HZ_EODD = -2
HZ_ENOMATERIAL = -3
HZ_ENOTSPD = -4
HZ_EWORKSPACE = -5
HZ_EHIP = -6
HZ_EDIVERGED = -7

HZ_FP64 = 0
HZ_FP32_REFINE = 1

HZ_GREEN_TETRA = 0
HZ_GREEN_ROTATED = 1
HZ_GREEN_CONTINUOUS = 2

HZ_SCHEME_AUTO = 0
HZ_SCHEME_SPECTRAL = 1
HZ_SCHEME_STENCIL = 2
HZ_SCHEME_STRAIN = 3

HZ_LOAD_STRAIN = 0
HZ_LOAD_STRESS = 1


class hz_opts(ctypes.Structure):
    _fields_ = [
        ("tol", c_double),
        ("max_iters", c_int32),
        ("precision", c_int32),
        ("ref_mode", c_int32),
        ("ref_C", c_double * 36),
        ("fixed_iters", c_int32),
        ("check_every", c_int32),
        ("trace_residual", POINTER(c_double)),
        ("trace_mean", POINTER(c_double)),
        ("inner_rho", c_double),
        ("inner_max", c_int32),
        ("scheme", c_int32),
        ("loading", c_int32),
        ("u_init", POINTER(c_double)),
        ("Ebar_init", POINTER(c_double)),
        ("fields_on_device", c_int32),
        ("green", c_int32),
    ]


class hz_info(ctypes.Structure):
    _fields_ = [
        ("status", c_int32),
        ("iters", c_int32),
        ("outer_rounds", c_int32),
        ("precision_used", c_int32),
        ("residual", c_double),
        ("seconds", c_double),
        ("seconds_to_1e6", c_double),
        ("wall_seconds", c_double),
        ("Ebar", c_double * 6),
    ]


# name -> (restype, argtypes); every entry point declared in include/hz.h
SIGNATURES = {
    "hz_default_opts": (None, [POINTER(hz_opts)]),
    "hz_create_grid": (c_int32, [c_int32, c_int32, c_int32, POINTER(c_void_p)]),
    "hz_set_material": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_uint16)]),
    "hz_set_eigenstrain": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "hz_workspace_bytes": (c_int64, [c_void_p, c_int32, c_int32]),
    "hz_bind_workspace": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_int32]),
    "hz_solve": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(hz_opts), POINTER(c_double),
                           POINTER(c_double), POINTER(c_double), POINTER(hz_info)]),
    "hz_solve_static": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(c_double), POINTER(hz_opts),
                                  POINTER(c_double), POINTER(c_double), POINTER(c_double), POINTER(hz_info)]),
    "hz_effective_stiffness": (c_int32, [c_void_p, POINTER(hz_opts), POINTER(c_double), POINTER(hz_info)]),
    "hz_get_displacement": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "hz_reference_medium": (c_int32, [c_int32, POINTER(c_double), POINTER(c_double)]),
    "hz_scheme_available": (c_int32, [c_void_p, c_int32]),
    "hz_profile": (c_int32, [c_void_p, c_int32]),
    "hz_profile_read": (c_int32, [c_void_p, c_int32, POINTER(c_char_p), POINTER(c_double), POINTER(c_int64)]),
    "hz_destroy_grid": (None, [c_void_p]),
    "hz_last_error": (c_char_p, []),
    "hz_server_bytes": (c_int64, [c_int32]),
    "hz_request_bytes": (c_int64, [c_void_p, c_int32, c_int32]),
    "hz_server_create": (c_int32, [c_void_p, c_int64, c_void_p, c_int32, c_int32, POINTER(c_void_p)]),
    "hz_server_submit": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(c_double), POINTER(hz_opts),
                                   POINTER(c_int64)]),
    "hz_server_step": (c_int32, [c_void_p, POINTER(c_int32)]),
    "hz_server_query": (c_int32, [c_void_p, c_int64, POINTER(c_double), POINTER(hz_info)]),
    "hz_server_release": (c_int32, [c_void_p, c_int64]),
    "hz_server_pending": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "hz_server_set_streams": (c_int32, [c_void_p, c_int32]),
    "hz_server_destroy": (None, [c_void_p]),
}

_lib = None


def load():
    """Load libhz.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is missing: build it with `python -m paper_2405_11168_amd.build`"
            " (or __graft_entry__.build()); there is no CPU fallback")
    # PyTorch ships its own HIP runtime.  Importing it first makes the dynamic
    # loader satisfy libhz.so's libamdhip64.so.7 / libhsa-runtime64.so.1 with the
    # copies torch already loaded (same SONAMEs), so the process has a single HIP
    # runtime and the torch-owned workspace is valid for the library's kernels.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hz error {code}: {msg}")
        self.code = code


def check(rc):
    if rc < 0:
        raise HzError(rc, load().hz_last_error().decode())
    return rc

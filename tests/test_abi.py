"""C ABI: the library loads, exports every declared symbol, and its host-only
logic (argument checks, sizes, workspace layout, reference-medium rule) works
without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import hz_synth as syn
import paper_2405_11168_amd as hz
from paper_2405_11168_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hz.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(hz_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = hz.lib()
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.SIGNATURES, n


def test_size_checks():
    lib = hz.lib()
    h = ctypes.c_void_p()
    assert lib.hz_create_grid(16, 16, 15, ctypes.byref(h)) == _abi.HZ_EODD
    assert lib.hz_create_grid(22, 16, 16, ctypes.byref(h)) == _abi.HZ_EINVAL  # prime 11
    assert lib.hz_create_grid(0, 16, 16, ctypes.byref(h)) == _abi.HZ_EINVAL
    assert lib.hz_create_grid(16, 16, 16, None) == _abi.HZ_EINVAL
    assert b"NULL" in lib.hz_last_error()
    for shape in [(2, 2, 2), (6, 10, 14), (320, 192, 192), (256, 256, 256)]:
        g = hz.Grid(*shape)
        assert g.workspace_bytes(hz.HZ_FP64, 1) > 0


def test_size_limits_and_both_schemes_on_every_accepted_grid():
    """Each axis up to the largest 7-smooth even size whose FP64 transform tile fits the
    LDS the transforms use (64 KB for x and y: N1 <= 1008, N2 <= 2016; 68 KB for z:
    N3 <= 1080), a load's 12 spectra under
    2^31 complex elements (700^3 accepted, 720^3 refused); on every accepted grid both
    forms are available, the stencil form's x transforms splitting on an odd radix, or in
    one pass, where N1/2 has no factor 2."""
    lib = hz.lib()
    h = ctypes.c_void_p()
    for shape, code in [((1008, 8, 8), hz.HZ_OK), ((1024, 8, 8), _abi.HZ_EINVAL),
                        ((8, 2016, 8), hz.HZ_OK), ((8, 2048, 8), _abi.HZ_EINVAL),
                        ((8, 8, 1080), hz.HZ_OK), ((8, 8, 1120), _abi.HZ_EINVAL),
                        ((700, 700, 700), hz.HZ_OK), ((720, 720, 720), _abi.HZ_EINVAL)]:
        assert lib.hz_create_grid(*shape, ctypes.byref(h)) == code, shape
        if code == hz.HZ_OK:
            lib.hz_destroy_grid(h)
    for shape in [(2, 4, 6), (6, 10, 12), (10, 6, 8), (14, 8, 28), (18, 20, 6), (30, 12, 10),
                  (126, 8, 6), (128, 128, 128), (1008, 8, 8), (192, 192, 320)]:
        g = hz.Grid(*shape)
        assert g.scheme_available(hz.HZ_SCHEME_SPECTRAL) and g.scheme_available(hz.HZ_SCHEME_STENCIL), shape


def test_material_validation():
    g = hz.Grid(4, 4, 6)
    C = np.stack([syn.isotropic_voigt(1, 0.3), syn.isotropic_voigt(2, 0.3)])
    ph = np.zeros((6, 4, 4), dtype=np.uint16)
    g.set_material(C, ph)
    bad = C.copy()
    bad[1, 0, 0] = -5.0
    with pytest.raises(hz.HzError) as e:
        g.set_material(bad, ph)
    assert e.value.code == _abi.HZ_ENOTSPD
    ph2 = ph.copy()
    ph2[0, 0, 0] = 7
    with pytest.raises(hz.HzError) as e:
        g.set_material(C, ph2)
    assert e.value.code == _abi.HZ_EINVAL
    # voids (zero stiffness) are accepted
    C0 = C.copy()
    C0[1] = 0.0
    g.set_material(C0, ph)


def test_solve_without_workspace_is_rejected():
    lib = hz.lib()
    h = ctypes.c_void_p()
    assert lib.hz_create_grid(4, 4, 4, ctypes.byref(h)) == 0
    o = _abi.hz_opts()
    lib.hz_default_opts(ctypes.byref(o))
    E = np.zeros(6)
    rc = lib.hz_solve(h, 1, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o), None, None,
                      None, None)
    assert rc == _abi.HZ_ENOMATERIAL
    C = syn.isotropic_voigt(1, 0.3)
    ph = np.zeros(64, dtype=np.uint16)
    assert lib.hz_set_material(h, 1, C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))) == 0
    rc = lib.hz_solve(h, 1, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o), None, None,
                      None, None)
    assert rc == _abi.HZ_EWORKSPACE
    lib.hz_destroy_grid(h)


def test_workspace_scales_with_loads_and_precision():
    g = hz.Grid(64, 48, 40)
    a1 = g.workspace_bytes(hz.HZ_FP64, 1)
    a6 = g.workspace_bytes(hz.HZ_FP64, 6)
    S = (64 // 2 + 1) * 48 * 40
    # per load: 12 spectra + 2 displacement buffers, FP64 complex (+ small status blocks)
    per = (12 + 6) * S * 16
    assert per <= (a6 - a1) / 5 < 1.02 * per
    r1 = g.workspace_bytes(hz.HZ_FP32_REFINE, 1)
    r2 = g.workspace_bytes(hz.HZ_FP32_REFINE, 2)
    per = (12 * 16 + 6 * 8 + 3 * 16 + 3 * 8) * S
    assert per <= r2 - r1 < 1.02 * per


def test_reference_medium_rule():
    """Automatic reference: isotropic, nu0 = 0, Mandel modulus at the midpoint of the
    extreme Mandel eigenvalues over all phases."""
    rng = np.random.default_rng(0)
    C = np.stack([syn.random_spd_voigt(rng, 0.5, 3.0), syn.random_spd_voigt(rng, 2.0, 40.0)])
    s = np.array([1, 1, 1, 2 ** .5, 2 ** .5, 2 ** .5])
    ev = np.concatenate([np.linalg.eigvalsh(c * np.outer(s, s)) for c in C])
    m = 0.5 * (ev.min() + ev.max())
    C0 = hz.reference_medium(C)
    expect = np.diag([m, m, m, m / 2, m / 2, m / 2])
    assert np.abs(C0 - expect).max() < 1e-10 * m


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of hz_opts / hz_info have the C compiler's sizes and offsets."""
    fields = {"hz_opts": [f[0] for f in _abi.hz_opts._fields_], "hz_info": [f[0] for f in _abi.hz_info._fields_]}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hz.h"', "int main(void) {"]
    for st, names in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for n in names:
            lines.append(f'  printf("{st}.{n} %zu\\n", offsetof({st}, {n}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for st, cls in (("hz_opts", _abi.hz_opts), ("hz_info", _abi.hz_info)):
        assert int(out[st]) == ctypes.sizeof(cls), st
        for n in fields[st]:
            assert int(out[f"{st}.{n}"]) == getattr(cls, n).offset, (st, n)


def test_eigenstrain_and_loading_validation():
    lib = hz.lib()
    g = hz.Grid(4, 4, 6)
    e0 = np.zeros((2, 6))
    with pytest.raises(hz.HzError) as e:
        g.set_eigenstrain(e0)
    assert e.value.code == _abi.HZ_ENOMATERIAL
    C = np.stack([syn.isotropic_voigt(1, 0.3), syn.isotropic_voigt(2, 0.3)])
    g.set_material(C, np.zeros((6, 4, 4), dtype=np.uint16))
    with pytest.raises(hz.HzError) as e:
        g.set_eigenstrain(np.zeros((3, 6)))  # one row per phase
    assert e.value.code == _abi.HZ_EINVAL
    e0[1, 2] = np.nan
    with pytest.raises(hz.HzError) as e:
        g.set_eigenstrain(e0)
    assert e.value.code == _abi.HZ_EINVAL
    e0[1, 2] = 0.01
    g.set_eigenstrain(e0)
    g.set_eigenstrain(None)
    # option checks come before the workspace check, so they run without a device
    E = np.zeros(6)
    for prec, loading in ((hz.HZ_FP32_REFINE, hz.HZ_LOAD_STRESS), (hz.HZ_FP64, 7)):
        o = hz._opts(precision=prec, loading=loading)
        rc = lib.hz_solve(g._h, 1, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o), None, None,
                          None, None)
        assert rc == _abi.HZ_EINVAL, (prec, loading)
    o = hz._opts(loading=hz.HZ_LOAD_STRESS)
    Ce = np.zeros(36)
    assert lib.hz_effective_stiffness(g._h, ctypes.byref(o), Ce.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      None) == _abi.HZ_EINVAL
    g.set_eigenstrain(e0)
    o = hz._opts()
    assert lib.hz_effective_stiffness(g._h, ctypes.byref(o), Ce.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      None) == _abi.HZ_EINVAL


def test_profile_modes():
    """hz_profile: 0 off, 1 every launch, 2 + i one entry of hz_profile_read; other
    values are rejected (host-side state only, no device needed)."""
    lib = _abi.load()
    g = hz.Grid(8, 8, 8)
    n = lib.hz_profile_read(g._h, 0, None, None, None)
    assert n > 0 and n % 2 == 0
    for mode in (1, 0, 2, 2 + n - 1, 0):
        assert lib.hz_profile(g._h, mode) == _abi.HZ_OK, mode
    for mode in (-1, 2 + n):
        assert lib.hz_profile(g._h, mode) == _abi.HZ_EINVAL, mode
    g.profile(True, only="stencil_f64")
    g.profile(False)
    with pytest.raises(ValueError):
        g.profile(True, only="no_such_kernel_f64")


def test_server_stream_count_checks_without_a_server():
    lib = hz.lib()
    assert lib.hz_server_set_streams(None, 2) == _abi.HZ_EINVAL
    assert b"NULL" in lib.hz_last_error()

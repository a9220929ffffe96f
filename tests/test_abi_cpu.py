"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every symbol include/lbm.h declares, its lattice tables equal the
oracle's element by element, and argument validation rejects bad input
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for must in ("lbm_create", "lbm_step", "lbm_macroscopic", "lbm_batch_step", "lbm_batch_create",
                 "lbm_get_populations", "lbm_set_populations", "lbm_invariants", "lbm_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(hiplib):
    L = hiplib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(hiplib.SYMBOLS) == declared_functions()


@pytest.mark.parametrize("q", (19, 27))
def test_kernel_tables_equal_oracle_tables(hiplib, orc, q):
    c, t, opp = hiplib.lattice(q)
    oc, ot, oopp = orc.lattice(q)
    assert np.array_equal(c, oc)
    assert np.array_equal(opp, oopp)
    assert np.abs(t - ot).max() <= 1e-17


def _desc(hiplib, **kw):
    d = hiplib.Desc()
    hiplib.lib().lbm_desc_default(ctypes.byref(d))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,needle", [
    ("lattice", 20, "lattice"), ("nx", 2, "dimensions"), ("omega", 2.0, "omega"), ("omega", 0.0, "omega"),
    ("scheme", 7, "scheme"), ("collision", 10, "collision"), ("storage_dtype", 5, "dtype"),
    ("omega3", 2.5, "omega3"), ("omega4", 2.0, "omega4"), ("omega_bulk", 2.0, "omega_bulk"),
    ("layout", 3, "layout"), ("block_size", 96, "block_size"), ("check_every", -1, "check_every"),
])
def test_invalid_descriptions_are_rejected(hiplib, field, value, needle):
    d = _desc(hiplib, **{field: value})
    out = (ctypes.c_size_t * 3)()
    assert hiplib.lib().lbm_required_bytes(ctypes.byref(d), out) == hiplib.EINVAL
    assert needle in hiplib.last_error()
    assert not hiplib.lib().lbm_create_ex(ctypes.byref(d))


def test_cumulant_model_is_d3q19_only(hiplib):
    d = _desc(hiplib, lattice=27, collision=9)
    out = (ctypes.c_size_t * 3)()
    assert hiplib.lib().lbm_required_bytes(ctypes.byref(d), out) == hiplib.EUNSUPPORTED
    assert "cumulant" in hiplib.last_error()
    d = _desc(hiplib, lattice=19, collision=9, omega3=1.5, omega4=0.5)
    assert hiplib.lib().lbm_required_bytes(ctypes.byref(d), out) == 0


def test_fast_lid_is_rejected(hiplib):
    assert not hiplib.lib().lbm_create(19, 8, 8, 8, 2, 0, 1.0, 0.5, 0)
    assert "lid" in hiplib.last_error()


@pytest.mark.parametrize("scheme,dtype,layout", [(0, 0, 0), (2, 1, 0), (1, 2, 1), (3, 0, 0), (3, 2, 1)])
def test_required_bytes(hiplib, scheme, dtype, layout):
    d = _desc(hiplib, nx=10, ny=11, nz=12, scheme=scheme, storage_dtype=dtype, layout=layout)
    out = (ctypes.c_size_t * 3)()
    assert hiplib.lib().lbm_required_bytes(ctypes.byref(d), out) == 0
    n = 10 * 11 * 12
    s = (8, 4, 2)[dtype]
    if layout == 0:   # SoA: streams of `stride` cells (room for the largest padding) plus a halo at both ends
        stride = (n + 1023) // 1024 * 1024 + 3072
        halo = (11 * 12 + 12 + 1 + 255) // 256 * 256
        assert out[0] == (19 * stride + 2 * halo) * s
    else:
        assert out[0] == 19 * n * s
    assert out[1] == (out[0] if scheme in (0, 3) else 0)   # 2Pop and 2Pop pull hold two arrays
    assert out[2] == n


def test_null_handles_are_rejected(hiplib):
    L = hiplib.lib()
    assert L.lbm_step(None, 1) == hiplib.EINVAL
    assert L.lbm_sync(None) == hiplib.EINVAL
    assert L.lbm_batch_step(None, 1) == hiplib.EINVAL
    assert not L.lbm_batch_create(0, None, 2, 0, 0, None)
    L.lbm_destroy(None)
    L.lbm_batch_destroy(None)


def test_batch_rejects_swap_and_unknown_schemes(hiplib):
    """The ensemble runs 2Pop, AA or 2Pop pull; swap is a valid scheme it does
    not support, 7 no scheme at all (checked before any device call)."""
    L = hiplib.lib()
    arr = (hiplib.CavityDesc * 1)()
    arr[0].nx = arr[0].ny = arr[0].nz = 16
    arr[0].omega, arr[0].u_lid, arr[0].trt_lambda = 1.8, 0.03, 0.25
    assert not L.lbm_batch_create(1, arr, hiplib.SCHEMES["swap"], 1, 1, None)
    assert "batch schemes" in hiplib.last_error()
    assert not L.lbm_batch_create(1, arr, 7, 1, 1, None)
    assert "batch schemes" in hiplib.last_error()


def test_batch_rejects_bad_launch_shapes(hiplib):
    """Fixed launch shapes outside what the fast kernel supports are refused
    before any device call."""
    L = hiplib.lib()
    arr = (hiplib.CavityDesc * 1)()
    arr[0].nx = arr[0].ny = arr[0].nz = 16
    arr[0].omega, arr[0].u_lid, arr[0].trt_lambda = 1.8, 0.03, 0.25
    for kw, msg in (({"block_size": 96}, "block_size"), ({"cells_per_thread": 3}, "cells_per_thread"),
                    ({"waves_per_simd": 9}, "waves_per_simd"), ({"xcd_split": 3}, "xcd_split")):
        o = hiplib.BatchOpts()
        for k, v in kw.items():
            setattr(o, k, v)
        assert not L.lbm_batch_create(1, arr, hiplib.SCHEMES["aa"], 1, 1, ctypes.byref(o))
        assert msg in hiplib.last_error()


@pytest.mark.parametrize("scheme", (0, 3))
def test_undersized_or_misaligned_caller_buffers_are_rejected(hiplib, scheme):
    """Caller buffers smaller than lbm_required_bytes reports, or not 256-byte
    aligned, are refused before any device work (the pointers below are never
    dereferenced: creation stops at the check)."""
    L = hiplib.lib()
    d = _desc(hiplib, nx=10, ny=11, nz=12, scheme=scheme)
    req = (ctypes.c_size_t * 3)()
    assert L.lbm_required_bytes(ctypes.byref(d), req) == 0
    fake = 1 << 40   # 256-byte aligned, never touched
    cases = [("pop", "pop_bytes", req[0]), ("flags", "flags_bytes", req[2]), ("out", "out_bytes", req[1])]
    for ptr, size, need in cases:
        d = _desc(hiplib, nx=10, ny=11, nz=12, scheme=scheme)
        setattr(d, ptr, fake)
        setattr(d, size, need - 1)
        assert not L.lbm_create_ex(ctypes.byref(d))
        assert f"caller buffer {ptr} holds {need - 1} bytes, {need} needed" in hiplib.last_error()
        d = _desc(hiplib, nx=10, ny=11, nz=12, scheme=scheme)
        setattr(d, ptr, fake + 64)
        setattr(d, size, need)
        assert not L.lbm_create_ex(ctypes.byref(d))
        assert "256-byte aligned" in hiplib.last_error()
    # a buffer given without its size is refused as well
    d = _desc(hiplib, nx=10, ny=11, nz=12, scheme=scheme, pop=fake)
    assert not L.lbm_create_ex(ctypes.byref(d))
    assert "caller buffer pop holds 0 bytes" in hiplib.last_error()

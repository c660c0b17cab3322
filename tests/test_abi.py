"""Host-side checks of the C ABI (no GPU needed).

The library must build, load and export every function include/ffpat.h
declares; argument validation must reject bad input before touching any
device memory (so these calls are safe without a GPU).
"""
import ctypes
import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffpat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffpat_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1901_06503_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1901_06503_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["ffpat_forward", "ffpat_adjoint", "ffpat_reconstruct", "ffpat_plan_create",
                     "ffpat_plan_destroy", "ffpat_workspace_bytes", "ffpat_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_1901_06503_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_version(lib):
    assert b"gfx950" in lib.ffpat_version()


def _geom(nx=32, ny=30, nz=20, dx=0.05, T=0.5, cfl=0.3, n_angles=16, ns=0, ds=0.0, dtype=0, ndim=3,
          angles=None, flags=0):
    from paper_1901_06503_amd import _lib
    ang = np.linspace(0, math.pi, n_angles, endpoint=False) if angles is None else np.asarray(angles, float)
    g = _lib.Geom(nx, ny, nz, ndim, dx, T, cfl, n_angles, ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  ns, ds, dtype, flags)
    return g, ang


def test_workspace_bytes_accounts_for_all_buffers(lib):
    g, _a = _geom(nx=64, ny=64, nz=64, n_angles=64)
    out = ctypes.c_size_t()
    assert lib.ffpat_workspace_bytes(ctypes.byref(g), ctypes.byref(out)) == 0
    nvox, ndat = 64 ** 3, 64 ** 3
    padded = 2 * 64 * 64 * (64 + 6) + 64 * 64 * (64 + 5)   # line copies (plane, transpose) + detector rows
    need = (7 * nvox + ndat + padded) * 4                  # k' + six volumes
    assert need <= out.value < need + 2 * 1024 * 1024
    g64, _b = _geom(nx=64, ny=64, nz=64, n_angles=64, dtype=1)
    out64 = ctypes.c_size_t()
    assert lib.ffpat_workspace_bytes(ctypes.byref(g64), ctypes.byref(out64)) == 0
    assert out64.value > 1.9 * out.value


@pytest.mark.parametrize("kw,status", [
    (dict(cfl=0.5), -2), (dict(cfl=0.7), -2), (dict(cfl=-0.1), -2),
    (dict(cfl=0.6, ndim=2), 0), (dict(cfl=0.62, ndim=2), -2),
    (dict(nx=0), -1), (dict(dx=0.0), -1), (dict(dx=float("nan")), -1), (dict(T=-1.0), -1),
    (dict(n_angles=0), -1), (dict(ns=-3), -1), (dict(ds=-1.0), -1), (dict(dtype=7), -6), (dict(ndim=4), -1),
    (dict(angles=[0.0, float("inf")], n_angles=2), -1),
    (dict(flags=4), 0), (dict(flags=8), 0), (dict(flags=32), 0), (dict(flags=4 | 8), -1), (dict(flags=4 | 32), -1),
    (dict(flags=8 | 32), -1), (dict(flags=16), -1), (dict(flags=1 << 31), -1),
])
def test_geometry_validation(lib, kw, status):
    g, _a = _geom(**kw)
    out = ctypes.c_size_t()
    assert lib.ffpat_workspace_bytes(ctypes.byref(g), ctypes.byref(out)) == status
    if status != 0:
        assert lib.ffpat_last_error() != b""


@pytest.mark.parametrize("nx,ny,dtype,status", [
    (32768, 32768, 0, -1),          # padded FP32 plane 4.3e9 bytes: offsets would wrap
    (32762, 32768, 0, -1),          # 32762 + 6 columns: exactly 2^32 bytes
    (32761, 32768, 0, 0),           # just below
    (23170, 23170, 1, -1),          # FP64: 23170 x 23176 x 8 > 2^32
    (23000, 23000, 1, 0),
    (1, 1 << 30, 0, -1),            # the transposed copy's lines are the long ones
])
def test_planes_too_large_for_32_bit_projector_offsets(lib, nx, ny, dtype, status):
    """X (eq. Radon) addresses a padded plane with 32-bit byte offsets: geometries
    whose padded plane reaches 2^32 bytes are rejected on the host."""
    g, _a = _geom(nx=nx, ny=ny, nz=1, n_angles=4, ns=64, dtype=dtype)
    out = ctypes.c_size_t()
    assert lib.ffpat_workspace_bytes(ctypes.byref(g), ctypes.byref(out)) == status
    if status:
        assert b"2^32" in lib.ffpat_last_error()


def test_plan_create_rejects_before_device_work(lib):
    # invalid geometry with a non-null dummy pointer: rejected on the host, nothing dereferenced
    g, _a = _geom(cfl=0.9)
    plan = ctypes.c_void_p()
    rc = lib.ffpat_plan_create(ctypes.byref(g), ctypes.c_void_p(0x1000), None, ctypes.byref(plan))
    assert rc == -2 and not plan.value
    g2, _b = _geom()
    rc = lib.ffpat_plan_create(ctypes.byref(g2), None, None, ctypes.byref(plan))
    assert rc == -1 and b"c_dev" in lib.ffpat_last_error()


def test_null_plan_is_rejected(lib):
    for name in ["ffpat_forward", "ffpat_adjoint", "ffpat_wave", "ffpat_wave_adjoint", "ffpat_project",
                 "ffpat_backproject", "ffpat_ramp"]:
        assert getattr(lib, name)(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -1
    i32 = ctypes.c_int32()
    assert lib.ffpat_plan_steps_per_pass(None, ctypes.byref(i32)) == -1
    assert lib.ffpat_plan_stencil_shape(None, ctypes.byref(i32), None, None) == -1
    assert lib.ffpat_plan_set_speed(None, ctypes.c_void_p(16), None) == -1
    assert lib.ffpat_plan_destroy(None) == 0


def test_plain_c_caller_builds_links_and_runs(lib, tmp_path):
    # the boundary is C: a C99 program compiled with -pedantic against the header links
    # the library and gets the documented statuses from the calls that need no device
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    from paper_1901_06503_amd import _lib
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = str(tmp_path / "abi_consumer")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I" + os.path.dirname(HEADER),
                    os.path.join(ROOT, "tests", "abi_consumer.c"), "-L" + libdir, "-lffpat",
                    "-Wl,-rpath," + libdir, "-o", exe], check=True)
    run = subprocess.run([exe], capture_output=True, text=True)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.count("ok ") == 9


def test_stream_probe_library_rejects_bad_arguments_before_launching(lib):
    # the streaming-ceiling kernels the benchmark times live in their own library
    from paper_1901_06503_amd import build
    probe = ctypes.CDLL(build.PROBE_LIB)
    f = probe.ffpat_probe_stream
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    p16 = ctypes.c_void_p(0x1000)
    assert f(0, p16, None, p16, p16, p16, 1024, 64, None) == -1          # b missing
    assert f(1, p16, None, None, None, None, 1022, 64, None) == -1       # not a multiple of 4
    assert f(1, ctypes.c_void_p(0x1004), None, None, p16, None, 1024, 64, None) == -1   # misaligned
    assert f(1, p16, None, None, p16, None, 1024, 0, None) == -1         # no work-groups
    assert f(2, p16, p16, p16, p16, p16, 1024, 64, None) == -1           # unknown pattern


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1901_06503_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()

"""FP64 CPU oracle (test infrastructure only).

Plain double-precision implementation of the one-step full-field PAT path
(Haltmeier, Zangerl, Nuster, Nguyen 2019): the wave operator W_T (Sec. 2.1,
eq. wave1/wave2, eq. Wo), its Euclidean transpose (Sec. 3.1), the plane-wise
X-ray transform X (eq. Radon) and its transpose, the ramp preconditioner
Lambda (Sec. 3.1), and Algorithm 8 (Sec. 3.2) with its power-iteration step.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library.

Parity status: every function here is pinned by CPU tests against closed
forms, invariants or brute force (tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffpat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

POSITIVITY = 1
PRECOND = 2
REG_GRAD = 4


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c99", "-D_DEFAULT_SOURCE", "-shared",
                               "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """Compiles the oracle with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
    -O1 -g, errors fatal) into `path`, for the CPU tests' sanitizer run; the process
    that loads it preloads gcc's sanitizer runtimes."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-std=c99", "-D_DEFAULT_SOURCE", "-shared", "-fPIC",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           _SRC, "-o", path, "-lm"])
    return path


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ndim", ctypes.c_int32), ("dx", ctypes.c_double), ("T", ctypes.c_double),
                ("cfl", ctypes.c_double), ("n_angles", ctypes.c_int32),
                ("angles", ctypes.POINTER(ctypes.c_double)), ("ns", ctypes.c_int32),
                ("ds", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("FFPAT_ORACLE_LIB")   # the sanitizer build, in the CPU tests' sanitizer run
        if not path:
            build()
            path = _LIB
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        G = ctypes.POINTER(_Geom)
        for name, args, res in [
            ("orc_time_grid", [ctypes.c_double] * 4 + [P, P], ctypes.c_int),
            ("orc_laplacian", [G, P, P], None),
            ("orc_neg_lap7", [G, P, P], None),
            ("orc_wave", [G, P, P, P], ctypes.c_int),
            ("orc_wave_T", [G, P, P, P], ctypes.c_int),
            ("orc_project", [G, P, P], None),
            ("orc_backproject", [G, P, P], None),
            ("orc_ramp", [G, P, P], None),
            ("orc_ramp_scale", [G], ctypes.c_double),
            ("orc_ramlak_tap", [ctypes.c_long], ctypes.c_double),
            ("orc_forward", [G, P, P, P], ctypes.c_int),
            ("orc_adjoint", [G, P, P, P], ctypes.c_int),
            ("orc_power", [G, P, ctypes.c_uint32, P, ctypes.c_int32, P, P], ctypes.c_int),
            ("orc_fb", [G, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                        ctypes.c_uint32, P, P, P, P, P], ctypes.c_int),
            ("orc_prox_grad", [G, ctypes.c_double, P, P, ctypes.c_double, ctypes.c_int32], ctypes.c_int),
            ("orc_energy", [G, P, P, P], ctypes.c_double),
            ("orc_wave_history", [G, P, P, ctypes.c_int32, P], ctypes.c_int),
            ("orc_plan_info", [G, P, P, P, P], ctypes.c_int),
            ("orc_fbp", [G, P, P], ctypes.c_int),
            ("orc_fb_two_step", [G, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_uint32, P, P, P, P], ctypes.c_int),
        ]:
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


@dataclass
class Geometry:
    """Grid, time and detector geometry (volumes [nz][ny][nx], data [angle][z][s])."""
    nx: int
    ny: int
    nz: int
    dx: float
    T: float
    angles: np.ndarray
    cfl: float = 0.3
    ns: int = 0
    ds: float = 0.0
    ndim: int = 3
    _angles_c: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)
        if self.ns <= 0:
            self.ns = self.nx
        if self.ds <= 0:
            self.ds = self.dx

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def data_shape(self):
        return (len(self.angles), self.nz, self.ns)

    def _c(self):
        self._angles_c = np.ascontiguousarray(self.angles, dtype=np.float64)
        g = _Geom(self.nx, self.ny, self.nz, self.ndim, self.dx, self.T, self.cfl,
                  len(self._angles_c), self._angles_c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  self.ns, self.ds)
        return ctypes.byref(g), g


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _u8(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.shape != tuple(shape):
        raise ValueError(f"expected mask shape {tuple(shape)}, got {a.shape}")
    return a


def _p(a):
    return None if a is None else a.ctypes.data


def time_grid(T, cmax, cfl, dx):
    """(n_t, dt): dt = cfl dx / c_max rounded so that n_t dt = T."""
    lib = _load()
    nt = ctypes.c_int32()
    dt = ctypes.c_double()
    lib.orc_time_grid(T, cmax, cfl, dx, ctypes.addressof(nt), ctypes.addressof(dt))
    return nt.value, dt.value


def plan_info(geom: Geometry, c):
    lib = _load()
    c = _f64(c, geom.vol_shape)
    gp, _g = geom._c()
    nt = ctypes.c_int32(); dt = ctypes.c_double(); cm = ctypes.c_double()
    lib.orc_plan_info(gp, _p(c), ctypes.addressof(nt), ctypes.addressof(dt), ctypes.addressof(cm))
    return nt.value, dt.value, cm.value


def laplacian(geom: Geometry, f):
    lib = _load()
    f = _f64(f, geom.vol_shape)
    out = np.empty_like(f)
    gp, _g = geom._c()
    lib.orc_laplacian(gp, _p(f), _p(out))
    return out


def neg_lap7(geom: Geometry, f):
    lib = _load()
    f = _f64(f, geom.vol_shape)
    out = np.empty_like(f)
    gp, _g = geom._c()
    lib.orc_neg_lap7(gp, _p(f), _p(out))
    return out


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")


def wave(geom: Geometry, c, h):
    """W_T h."""
    lib = _load()
    c = _f64(c, geom.vol_shape); h = _f64(h, geom.vol_shape)
    out = np.empty_like(h)
    gp, _g = geom._c()
    _check(lib.orc_wave(gp, _p(c), _p(h), _p(out)))
    return out


def wave_T(geom: Geometry, c, g):
    """W_T^T g (Euclidean transpose)."""
    lib = _load()
    c = _f64(c, geom.vol_shape); g = _f64(g, geom.vol_shape)
    out = np.empty_like(g)
    gp, _g = geom._c()
    _check(lib.orc_wave_T(gp, _p(c), _p(g), _p(out)))
    return out


def project(geom: Geometry, vol):
    """X vol -> data [angle][z][s]."""
    lib = _load()
    vol = _f64(vol, geom.vol_shape)
    out = np.empty(geom.data_shape)
    gp, _g = geom._c()
    lib.orc_project(gp, _p(vol), _p(out))
    return out


def backproject(geom: Geometry, data):
    """X^T data -> volume."""
    lib = _load()
    data = _f64(data, geom.data_shape)
    out = np.empty(geom.vol_shape)
    gp, _g = geom._c()
    lib.orc_backproject(gp, _p(data), _p(out))
    return out


def ramp(geom: Geometry, r):
    """Lambda r (row-wise Ram-Lak Toeplitz product, scaled)."""
    lib = _load()
    r = _f64(r, geom.data_shape)
    out = np.empty_like(r)
    gp, _g = geom._c()
    lib.orc_ramp(gp, _p(r), _p(out))
    return out


def ramp_scale(geom: Geometry) -> float:
    lib = _load()
    gp, _g = geom._c()
    return lib.orc_ramp_scale(gp)


def ramlak_tap(n: int) -> float:
    return _load().orc_ramlak_tap(int(n))


def forward(geom: Geometry, c, h):
    """A h = X W_T h."""
    lib = _load()
    c = _f64(c, geom.vol_shape); h = _f64(h, geom.vol_shape)
    out = np.empty(geom.data_shape)
    gp, _g = geom._c()
    _check(lib.orc_forward(gp, _p(c), _p(h), _p(out)))
    return out


def adjoint(geom: Geometry, c, data):
    """A^T data = W_T^T X^T data."""
    lib = _load()
    c = _f64(c, geom.vol_shape); data = _f64(data, geom.data_shape)
    out = np.empty(geom.vol_shape)
    gp, _g = geom._c()
    _check(lib.orc_adjoint(gp, _p(c), _p(data), _p(out)))
    return out


def power(geom: Geometry, c, n_power=20, flags=PRECOND, det_mask=None):
    """Power-iteration estimate of ||A^T chi Lambda chi A||; returns (L, history)."""
    lib = _load()
    c = _f64(c, geom.vol_shape)
    m = _u8(det_mask, geom.data_shape)
    L = ctypes.c_double()
    hist = np.zeros(n_power)
    gp, _g = geom._c()
    _check(lib.orc_power(gp, _p(c), flags, _p(m), n_power, ctypes.addressof(L), _p(hist)))
    return L.value, hist


def fb(geom: Geometry, c, G, lam, step=0.0, n_iter=5, n_power=20, flags=POSITIVITY | PRECOND,
       support=None, det_mask=None, h0=None):
    """Algorithm 8.  Returns (h_K, objective[K], step)."""
    lib = _load()
    c = _f64(c, geom.vol_shape); G = _f64(G, geom.data_shape)
    h = np.zeros(geom.vol_shape) if h0 is None else _f64(h0, geom.vol_shape).copy()
    sup = _u8(support, geom.vol_shape)
    m = _u8(det_mask, geom.data_shape)
    obj = np.zeros(max(n_iter, 1))
    s = ctypes.c_double()
    gp, _g = geom._c()
    _check(lib.orc_fb(gp, _p(c), _p(G), lam, step, n_iter, n_power, flags, _p(sup), _p(m), _p(h),
                      _p(obj), ctypes.addressof(s)))
    return h, obj[:n_iter], s.value


def prox_grad(geom: Geometry, tau, f, tol=1e-13, maxit=10000):
    """Solves (I + tau D^T D) h = f (prox of tau/2 ||D h||^2)."""
    lib = _load()
    f = _f64(f, geom.vol_shape)
    h = np.empty_like(f)
    gp, _g = geom._c()
    it = lib.orc_prox_grad(gp, tau, _p(f), _p(h), tol, maxit)
    if it < 0:
        raise RuntimeError("oracle prox_grad failed")
    return h


def energy(geom: Geometry, c, p0, p1):
    lib = _load()
    c = _f64(c, geom.vol_shape); p0 = _f64(p0, geom.vol_shape); p1 = _f64(p1, geom.vol_shape)
    gp, _g = geom._c()
    return lib.orc_energy(gp, _p(c), _p(p0), _p(p1))


def wave_history(geom: Geometry, c, h, nsteps):
    lib = _load()
    c = _f64(c, geom.vol_shape); h = _f64(h, geom.vol_shape)
    out = np.empty((nsteps + 1,) + geom.vol_shape)
    gp, _g = geom._c()
    _check(lib.orc_wave_history(gp, _p(c), _p(h), nsteps, _p(out)))
    return out


def fbp(geom: Geometry, G):
    """X^-1 G = X^T Lambda G (filtered backprojection per plane)."""
    lib = _load()
    G = _f64(G, geom.data_shape)
    out = np.empty(geom.vol_shape)
    gp, _g = geom._c()
    _check(lib.orc_fbp(gp, _p(G), _p(out)))
    return out


def fb_two_step(geom: Geometry, c, gvol, lam, step=0.0, n_iter=5, n_power=20, flags=POSITIVITY, support=None,
                h0=None):
    """Algorithm 9, second stage: FB on 1/2 ||W h - g||^2 + lambda R.  Returns (h_K, objective, step)."""
    lib = _load()
    c = _f64(c, geom.vol_shape); gvol = _f64(gvol, geom.vol_shape)
    h = np.zeros(geom.vol_shape) if h0 is None else _f64(h0, geom.vol_shape).copy()
    sup = _u8(support, geom.vol_shape)
    obj = np.zeros(max(n_iter, 1))
    s = ctypes.c_double()
    gp, _g = geom._c()
    _check(lib.orc_fb_two_step(gp, _p(c), _p(gvol), lam, step, n_iter, n_power, flags, _p(sup), _p(h), _p(obj),
                               ctypes.addressof(s)))
    return h, obj[:n_iter], s.value


def stripe_mask(geom: Geometry, a: float):
    """chi_M for M_theta = R minus [-a, a] (the central detector stripe is missing, Sec. 4)."""
    s = (np.arange(geom.ns) - 0.5 * (geom.ns - 1)) * geom.ds
    row = (np.abs(s) > a).astype(np.uint8)
    return np.ascontiguousarray(np.broadcast_to(row, geom.data_shape))

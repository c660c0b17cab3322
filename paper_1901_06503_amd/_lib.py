"""ctypes loader for libffpat.so (the C ABI declared in include/ffpat.h).

Argument marshalling only: every operator runs in the library's HIP kernels.
There is no fallback: if the library is missing the import of an operator
fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FFPAT_LIB_PATH selects another build of the same library (the CPU tests' sanitizer
# build); by default the in-tree libffpat.so
LIB_PATH = os.environ.get("FFPAT_LIB_PATH") or os.path.join(HERE, "libffpat.so")

OK, EINVAL, ECFL, ENOMEM, EHIP, EDIVERGED, EDTYPE, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {OK: "FFPAT_OK", EINVAL: "FFPAT_EINVAL", ECFL: "FFPAT_ECFL", ENOMEM: "FFPAT_ENOMEM",
                EHIP: "FFPAT_EHIP", EDIVERGED: "FFPAT_EDIVERGED", EDTYPE: "FFPAT_EDTYPE", EBUSY: "FFPAT_EBUSY"}
F32, F64 = 0, 1

PLAN_NAIVE_STENCIL = 1
PLAN_NO_GRAPHS = 2
PLAN_SINGLE_STEP = 4
PLAN_TWO_STEP = 8
PLAN_THREE_STEP = 32
POSITIVITY = 1
PRECOND = 2
REG_GRAD = 4
USE_PLAN_STEP = 8
TWO_STEP = 16


class FfpatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ndim", ctypes.c_int32), ("dx", ctypes.c_double), ("T", ctypes.c_double),
                ("cfl", ctypes.c_double), ("n_angles", ctypes.c_int32),
                ("angles", ctypes.POINTER(ctypes.c_double)), ("ns", ctypes.c_int32),
                ("ds", ctypes.c_double), ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FbParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("step", ctypes.c_double), ("n_iter", ctypes.c_int32),
                ("n_power", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("support", ctypes.c_void_p), ("det_mask", ctypes.c_void_p),
                ("objective", ctypes.POINTER(ctypes.c_double)), ("cg_tol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int32)]


_P = ctypes.c_void_p
SIGNATURES = {
    "ffpat_version": ([], ctypes.c_char_p),
    "ffpat_last_error": ([], ctypes.c_char_p),
    "ffpat_workspace_bytes": ([ctypes.POINTER(Geom), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ffpat_plan_create": ([ctypes.POINTER(Geom), _P, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "ffpat_plan_info": ([_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ffpat_plan_steps_per_pass": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "ffpat_plan_stencil_shape": ([_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "ffpat_plan_set_speed": ([_P, _P, _P], ctypes.c_int),
    "ffpat_plan_destroy": ([_P], ctypes.c_int),
    "ffpat_forward": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_adjoint": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_wave": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_wave_adjoint": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_project": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_backproject": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_ramp": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_fbp": ([_P, _P, _P, _P], ctypes.c_int),
    "ffpat_reconstruct": ([_P, _P, ctypes.POINTER(FbParams), _P, ctypes.POINTER(ctypes.c_double), _P],
                          ctypes.c_int),
    "ffpat_fb_enqueue": ([_P, _P, ctypes.POINTER(FbParams), _P, _P], ctypes.c_int),
    "ffpat_fb_enqueue_noalloc": ([_P, _P, ctypes.POINTER(FbParams), _P, _P], ctypes.c_int),
    "ffpat_fb_report": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _P],
                        ctypes.c_int),
}

_lib = None


def load():
    """Loads libffpat.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1901_06503_amd.build` "
                              "(the HIP library is required; there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(status: int):
    if status != OK:
        msg = load().ffpat_last_error().decode(errors="replace")
        raise FfpatError(status, msg)

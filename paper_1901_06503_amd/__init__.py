"""ffpat: one-step full-field photoacoustic reconstruction on AMD MI355X.

Python binding of libffpat (C ABI in include/ffpat.h).  Tensors are torch
device tensors used as plain device memory; every operator runs in the
library's HIP kernels on the caller's current stream.

Method: Haltmeier, Zangerl, Nuster, Nguyen, "Photoacoustic image
reconstruction from full field data in heterogeneous media" (2019):
forward operator A = X W_T (Problem 1, eq. fm), its transpose, the ramp
preconditioner (Sec. 3.1) and Algorithm 8 (Sec. 3.2).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import FfpatError, POSITIVITY, PRECOND, REG_GRAD, TWO_STEP, USE_PLAN_STEP

__all__ = ["Plan", "FfpatError", "ReconResult", "workspace_bytes", "version", "POSITIVITY", "PRECOND",
           "REG_GRAD", "TWO_STEP", "USE_PLAN_STEP"]


def version() -> str:
    return _lib.load().ffpat_version().decode()


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _make_geom(nx, ny, nz, dx, T, angles, ns, ds, cfl, ndim, dtype_code, flags):
    ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
    g = _lib.Geom(int(nx), int(ny), int(nz), int(ndim), float(dx), float(T), float(cfl), int(ang.size),
                  ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(ns), float(ds), int(dtype_code),
                  int(flags))
    return g, ang


def workspace_bytes(shape, dx, T, angles, ns=0, ds=0.0, cfl=0.3, ndim=3, dtype="float32") -> int:
    """Device bytes a plan of this geometry allocates (admission by HBM footprint)."""
    nz, ny, nx = shape
    code = _lib.F64 if str(dtype).endswith("64") else _lib.F32
    g, _keep = _make_geom(nx, ny, nz, dx, T, angles, ns, ds, cfl, ndim, code, 0)
    out = ctypes.c_size_t()
    _lib.check(_lib.load().ffpat_workspace_bytes(ctypes.byref(g), ctypes.byref(out)))
    return int(out.value)


@dataclass
class ReconResult:
    h: "object"            # torch tensor, h_K
    objective: np.ndarray  # J_0 .. J_{K-1} (FP64)
    step: float            # step size s used


class Plan:
    """Geometry + sound speed resident on one GPU, with the operators of the path.

    c: sound speed c(x) > 0 as a contiguous [nz][ny][nx] device tensor; its
    dtype (float32 or float64) sets the precision of every field.
    dx, T, angles, ns, ds, cfl, ndim: the geometry of ffpat_geom (ns = 0: nx bins,
    ds = 0: dx; ndim = 2: the z-invariant mode, every plane its own 2D problem).
    naive_stencil: the unblocked leapfrog kernel (for comparison).
    use_graphs: replay captured graphs in fb_enqueue / reconstruct.
    two_step_stencil: None lets the plan choose the leapfrog steps per stencil
    pass; True / False force two / one (FFPAT_PLAN_TWO_STEP / _SINGLE_STEP).
    stencil_steps: 1, 2 or 3 forces that many steps per pass where the grid allows
    (FFPAT_PLAN_SINGLE_STEP / _TWO_STEP / _THREE_STEP); excludes two_step_stencil.
    stream: torch stream (or None: the current one) for the plan's set-up.

    After creation: nt, dt, cmax (the time grid), steps_per_pass (1, 2 or 3 leapfrog
    steps per stencil pass) and stencil_shape (tile width, tile height, z-planes per
    work-group of that stencil kernel on this device; zeros for the naive kernel).
    """

    def __init__(self, c, dx, T, angles, ns=0, ds=0.0, cfl=0.3, ndim=3, naive_stencil=False, use_graphs=True,
                 two_step_stencil=None, stream=None, stencil_steps=None):
        torch = _torch()
        if not (isinstance(c, torch.Tensor) and c.is_cuda):
            raise TypeError("c must be a device tensor")
        if c.dtype not in (torch.float32, torch.float64):
            raise TypeError("c must be float32 or float64")
        if c.dim() != 3:
            raise ValueError("c must be [nz][ny][nx]")
        c = c.contiguous()
        self.dtype = c.dtype
        self.device = c.device
        nz, ny, nx = c.shape
        code = _lib.F64 if c.dtype == torch.float64 else _lib.F32
        if stencil_steps is not None and two_step_stencil is not None:
            raise ValueError("stencil_steps and two_step_stencil exclude each other")
        steps_flag = ({None: 0, True: _lib.PLAN_TWO_STEP, False: _lib.PLAN_SINGLE_STEP}[two_step_stencil]
                      if stencil_steps is None else
                      {1: _lib.PLAN_SINGLE_STEP, 2: _lib.PLAN_TWO_STEP, 3: _lib.PLAN_THREE_STEP}[stencil_steps])
        flags = ((_lib.PLAN_NAIVE_STENCIL if naive_stencil else 0) | (0 if use_graphs else _lib.PLAN_NO_GRAPHS)
                 | steps_flag)
        self._lib = _lib.load()
        g, self._angles = _make_geom(nx, ny, nz, dx, T, angles, ns, ds, cfl, ndim, code, flags)
        handle = ctypes.c_void_p()
        with torch.cuda.device(c.device):
            _lib.check(self._lib.ffpat_plan_create(ctypes.byref(g), ctypes.c_void_p(c.data_ptr()),
                                                   ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(handle)))
        self._h = handle
        self.shape = (nz, ny, nx)
        self.n_angles = int(self._angles.size)
        self.ns = int(ns) if ns else int(nx)
        self.data_shape = (self.n_angles, nz, self.ns)
        self.dx, self.T = float(dx), float(T)
        self.ds = float(ds) if ds else float(dx)
        nt = ctypes.c_int32(); dt = ctypes.c_double(); cm = ctypes.c_double()
        _lib.check(self._lib.ffpat_plan_info(self._h, ctypes.byref(nt), ctypes.byref(dt), ctypes.byref(cm)))
        self.nt, self.dt, self.cmax = nt.value, dt.value, cm.value
        sp = ctypes.c_int32()
        _lib.check(self._lib.ffpat_plan_steps_per_pass(self._h, ctypes.byref(sp)))
        self.steps_per_pass = sp.value          # 2 or 3: temporally blocked stencil kernel
        tx, ty, zc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.ffpat_plan_stencil_shape(self._h, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(zc)))
        self.stencil_shape = (tx.value, ty.value, zc.value)   # tile width, height, planes per work-group

    def set_speed(self, c, stream=None):
        """Replaces the sound speed (same shape and dtype) for a new problem of the same
        geometry, reusing the plan's memory: c_max, nt, dt and k' are recomputed and the
        stored step size is discarded (the next reconstruction runs its power iteration)."""
        torch = _torch()
        if not (isinstance(c, torch.Tensor) and c.is_cuda) or c.dtype != self.dtype or tuple(c.shape) != self.shape:
            raise TypeError(f"c must be a {self.dtype} device tensor of shape {self.shape}")
        c = c.contiguous()
        _lib.check(self._lib.ffpat_plan_set_speed(self._h, ctypes.c_void_p(c.data_ptr()),
                                                  ctypes.c_void_p(_stream_handle(stream))))
        nt = ctypes.c_int32(); dt = ctypes.c_double(); cm = ctypes.c_double()
        _lib.check(self._lib.ffpat_plan_info(self._h, ctypes.byref(nt), ctypes.byref(dt), ctypes.byref(cm)))
        self.nt, self.dt, self.cmax = nt.value, dt.value, cm.value

    # ------------------------------------------------------------------ helpers
    def _check_tensor(self, t, shape, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, plan on {self.device}")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, plan uses {self.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _empty(self, shape):
        return _torch().empty(shape, dtype=self.dtype, device=self.device)

    def _call(self, fn, src, src_shape, dst, dst_shape, stream, name):
        self._check_tensor(src, src_shape, name)
        if dst is None:
            dst = self._empty(dst_shape)
        self._check_tensor(dst, dst_shape, "out")
        _lib.check(fn(self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                      ctypes.c_void_p(_stream_handle(stream))))
        return dst

    # ------------------------------------------------------------------ operators
    def forward(self, h, out=None, stream=None):
        """g = X W_T h."""
        return self._call(self._lib.ffpat_forward, h, self.shape, out, self.data_shape, stream, "h")

    def adjoint(self, g, out=None, stream=None):
        """h = W_T^T X^T g."""
        return self._call(self._lib.ffpat_adjoint, g, self.data_shape, out, self.shape, stream, "g")

    def wave(self, h, out=None, stream=None):
        """p = W_T h."""
        return self._call(self._lib.ffpat_wave, h, self.shape, out, self.shape, stream, "h")

    def wave_adjoint(self, g, out=None, stream=None):
        """q = W_T^T g."""
        return self._call(self._lib.ffpat_wave_adjoint, g, self.shape, out, self.shape, stream, "g")

    def project(self, v, out=None, stream=None):
        """g = X v."""
        return self._call(self._lib.ffpat_project, v, self.shape, out, self.data_shape, stream, "v")

    def backproject(self, g, out=None, stream=None):
        """v = X^T g."""
        return self._call(self._lib.ffpat_backproject, g, self.data_shape, out, self.shape, stream, "g")

    def ramp(self, r, out=None, stream=None):
        """y = Lambda r."""
        return self._call(self._lib.ffpat_ramp, r, self.data_shape, out, self.data_shape, stream, "r")

    def fbp(self, G, out=None, stream=None):
        """vol = X^-1 G = X^T Lambda G (filtered backprojection per plane)."""
        return self._call(self._lib.ffpat_fbp, G, self.data_shape, out, self.shape, stream, "G")

    def landweber(self, G, n_iter, step=0.0, n_power=20, det_mask=None, h0=None, use_plan_step=False,
                  stream=None) -> ReconResult:
        """Algorithm 7, preconditioned Landweber: Algorithm 8 with R = 0 (no prox)."""
        return self.reconstruct(G, 0.0, n_iter, step=step, n_power=n_power, positivity=False, precond=True,
                                det_mask=det_mask, h0=h0, use_plan_step=use_plan_step, stream=stream)

    def stripe_mask(self, a):
        """chi_M for M_theta = R minus [-a, a]: 1 where the detector coordinate |s| > a."""
        torch = _torch()
        s = (torch.arange(self.ns, dtype=torch.float64) - 0.5 * (self.ns - 1)) * self.ds
        row = (s.abs() > a).to(torch.uint8)
        return row.expand(self.data_shape).contiguous().to(self.device)

    def _fb_params(self, G, lam, n_iter, step, n_power, positivity, precond, support, det_mask, h,
                   use_plan_step, objective, reg="l2", two_step=False, cg_tol=0.0, cg_maxit=0):
        self._check_tensor(G, self.shape if two_step else self.data_shape, "G")
        self._check_tensor(h, self.shape, "h")
        if reg not in ("l2", "grad"):
            raise ValueError("reg must be 'l2' (1/2||h||^2) or 'grad' (1/2||D h||^2)")
        flags = (POSITIVITY if positivity else 0) | (PRECOND if precond else 0)
        if reg == "grad":
            flags |= REG_GRAD
        if two_step:
            flags |= TWO_STEP
        if use_plan_step:
            flags |= USE_PLAN_STEP
        sup = 0
        if support is not None:
            self._check_mask(support, self.shape, "support")
            sup = support.data_ptr()
        msk = 0
        if det_mask is not None:
            self._check_mask(det_mask, self.data_shape, "det_mask")
            msk = det_mask.data_ptr()
        obj_ptr = objective.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if objective is not None else None
        return _lib.FbParams(float(lam), float(step), int(n_iter), int(n_power), flags,
                             ctypes.c_void_p(sup or None), ctypes.c_void_p(msk or None), obj_ptr,
                             float(cg_tol), int(cg_maxit))

    def reconstruct(self, G, lam, n_iter, step=0.0, n_power=20, positivity=True, precond=True,
                    support=None, det_mask=None, h0=None, use_plan_step=False, stream=None,
                    want_objective=True, reg="l2", two_step=False, cg_tol=0.0, cg_maxit=0) -> ReconResult:
        """Algorithm 8 (or Algorithm 9 with two_step=True and G = fbp(data)): K = n_iter
        forward-backward iterations from h0 (zeros by default; h0 is updated in place and
        returned as .h).  reg='grad' selects R = 1/2||D h||^2 (prox by conjugate gradients;
        positivity must be False).  Synchronises the stream at the end."""
        torch = _torch()
        h = torch.zeros(self.shape, dtype=self.dtype, device=self.device) if h0 is None else h0
        obj = np.zeros(max(int(n_iter), 1), dtype=np.float64)
        prm = self._fb_params(G, lam, n_iter, step, n_power, positivity, precond, support, det_mask, h,
                              use_plan_step, obj if want_objective else None, reg, two_step, cg_tol, cg_maxit)
        s = ctypes.c_double()
        _lib.check(self._lib.ffpat_reconstruct(self._h, ctypes.c_void_p(G.data_ptr()), ctypes.byref(prm),
                                               ctypes.c_void_p(h.data_ptr()), ctypes.byref(s),
                                               ctypes.c_void_p(_stream_handle(stream))))
        return ReconResult(h=h, objective=obj[:int(n_iter)], step=s.value)

    def fb_enqueue(self, G, lam, n_iter, h, step=0.0, n_power=20, positivity=True, precond=True, support=None,
                   det_mask=None, use_plan_step=False, stream=None, reg="l2", two_step=False, cg_tol=0.0,
                   cg_maxit=0):
        """Enqueues the step selection (unless use_plan_step or step > 0) and n_iter
        iterations on `stream` without host synchronisation (serving)."""
        prm = self._fb_params(G, lam, n_iter, step, n_power, positivity, precond, support, det_mask, h,
                              use_plan_step, None, reg, two_step, cg_tol, cg_maxit)
        _lib.check(self._lib.ffpat_fb_enqueue(self._h, ctypes.c_void_p(G.data_ptr()), ctypes.byref(prm),
                                              ctypes.c_void_p(h.data_ptr()),
                                              ctypes.c_void_p(_stream_handle(stream))))

    def fb_report(self, n=0, stream=None):
        """Waits for the stream; returns (step, objective[:n]) of the last enqueued run."""
        obj = np.zeros(max(int(n), 1), dtype=np.float64)
        s = ctypes.c_double()
        _lib.check(self._lib.ffpat_fb_report(self._h, ctypes.byref(s),
                                             obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if n else None,
                                             int(n), ctypes.c_void_p(_stream_handle(stream))))
        return s.value, obj[:int(n)]

    def _check_mask(self, m, shape, name):
        torch = _torch()
        if not isinstance(m, torch.Tensor) or not m.is_cuda or m.dtype != torch.uint8:
            raise TypeError(f"{name} must be a uint8 device tensor")
        if tuple(m.shape) != tuple(shape) or not m.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")
        if m.device != self.device:
            raise ValueError(f"{name} is on {m.device}, plan on {self.device}")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.ffpat_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

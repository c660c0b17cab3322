"""The no-allocation entry point ffpat_fb_enqueue_noalloc, through the C ABI.

Its work is ffpat_fb_enqueue's (Algorithm 8, Sec. 3.2) with the objective values
in the library's static per-device array and every kernel launched eagerly.  Two
calls in a row (the second on a smaller grid, fewer angles and iterations, the
other precision) must each give what ffpat_fb_enqueue gives on the same plan: the
same kernels in the same order, so iterate, step and objective values are
compared at the reconstruction tolerances and found equal bit for bit.  The
second call's values must be its own, not the first call's left in the array.
"""
import ctypes

import numpy as np
import pytest

from conftest import rel_l2, to_dev
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_ITER = 65536


def _problem(shape, n_angles, seed, dtype):
    import paper_1901_06503_amd as ff
    nz, ny, nx = shape
    dx = synth.grid_spacing(max(shape))
    rng = np.random.default_rng(seed)
    c = synth.sound_speed(shape, dx, rng, 2, 0.2, (0.8, 1.2))
    h = np.abs(synth.gaussian_smooth(synth.balls(shape, dx, rng, 4), 1.0))
    P = ff.Plan(to_dev(c, dtype), dx, 0.45, synth.uniform_angles(n_angles))
    g = P.forward(to_dev(h, dtype))
    noise = torch.from_numpy(rng.standard_normal(P.data_shape)).to(g.device, dtype)
    return P, g + 0.02 * float(g.double().mean()) * noise


def _run(P, G, n_iter, entry):
    """Enqueues through `entry` (a C ABI function), then ffpat_fb_report."""
    from paper_1901_06503_amd import _lib
    lib = _lib.load()
    h = torch.zeros(P.shape, dtype=P.dtype, device="cuda")
    prm = P._fb_params(G, 1e-3, n_iter, 0.0, 12, True, True, None, None, h, False, None)
    stream = torch.cuda.current_stream()
    _lib.check(entry(P._h, ctypes.c_void_p(G.data_ptr()), ctypes.byref(prm), ctypes.c_void_p(h.data_ptr()),
                     ctypes.c_void_p(stream.cuda_stream)))
    obj = np.zeros(n_iter, dtype=np.float64)
    step = ctypes.c_double()
    _lib.check(lib.ffpat_fb_report(P._h, ctypes.byref(step), obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   n_iter, ctypes.c_void_p(stream.cuda_stream)))
    return h, obj, step.value


def test_noalloc_enqueue_equals_enqueue_on_two_calls():
    from paper_1901_06503_amd import _lib
    lib = _lib.load()
    cases = [((20, 34, 40), 18, 5, torch.float32), ((9, 14, 16), 7, 3, torch.float64)]
    first_obj = None
    for shape, n_angles, n_iter, dtype in cases:
        print(f"[no-alloc] shape={shape} angles={n_angles} iterations={n_iter} {dtype}", flush=True)
        P, G = _problem(shape, n_angles, 71, dtype)
        with P:
            h_ref, obj_ref, s_ref = _run(P, G, n_iter, lib.ffpat_fb_enqueue)
            h, obj, s = _run(P, G, n_iter, lib.ffpat_fb_enqueue_noalloc)
        tol = 1e-4 if dtype == torch.float32 else 1e-10
        assert s == pytest.approx(s_ref, rel=tol)
        assert rel_l2(h.double().cpu().numpy(), h_ref.double().cpu().numpy()) <= tol
        assert np.allclose(obj, obj_ref, rtol=tol, atol=0)
        assert s == s_ref and torch.equal(h, h_ref) and np.array_equal(obj, obj_ref)
        assert np.all(np.isfinite(obj)) and obj[-1] < obj[0]
        if first_obj is not None:
            assert not np.array_equal(obj, first_obj[:len(obj)])
        first_obj = obj


def test_noalloc_enqueue_rejects_more_iterations_than_the_static_history():
    from paper_1901_06503_amd import _lib
    lib = _lib.load()
    P, G = _problem((6, 10, 12), 5, 72, torch.float64)
    with P:
        h = torch.zeros(P.shape, dtype=P.dtype, device="cuda")
        prm = P._fb_params(G, 1e-3, MAX_ITER + 1, 0.0, 4, True, True, None, None, h, False, None)
        rc = lib.ffpat_fb_enqueue_noalloc(P._h, ctypes.c_void_p(G.data_ptr()), ctypes.byref(prm),
                                          ctypes.c_void_p(h.data_ptr()), None)
        torch.cuda.synchronize()
        assert rc == _lib.EINVAL and b"65536" in lib.ffpat_last_error()
        assert not h.any()

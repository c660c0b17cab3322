"""GPU parity of the methods around the hot path (against the FP64 oracle):

* filtered backprojection X^-1 = X^* Lambda (Sec. 3.1);
* Algorithm 9 (two-step: FB on 1/2||W h - g||^2 with g = X^-1 G), l2 and
  gradient regularisers;
* Algorithm 8 with the paper's gradient regulariser R = 1/2 ||D h||^2 (prox
  by device-resident conjugate gradients);
* Algorithm 7 (preconditioned Landweber = Algorithm 8 with R = 0);
* limited data: the central detector stripe [-a, a] missing (Sec. 4);
* the z-invariant 2D mode under Algorithm 8.
"""
import math

import numpy as np
import pytest

from conftest import rel_l2, rounded, to_dev, to_np
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
TOL_FB = {F32: 1e-4, F64: 1e-10}


def _case(shape, seed, n_angles, dtype, T=0.4, ndim=3, ds_ratio=1.0):
    import oracle
    import paper_1901_06503_amd as ff
    nz, ny, nx = shape
    dx = synth.grid_spacing(max(nx, ny))
    ds = ds_ratio * dx
    ns = nx if ds_ratio == 1.0 else int(math.ceil(nx / ds_ratio)) + 4
    rng = np.random.default_rng(seed)
    c = rounded(synth.sound_speed(shape, dx, rng, 3, 0.2, (0.8, 1.2)), dtype)
    h = rounded(synth.gaussian_smooth(synth.balls(shape, dx, rng, 4), 1.0), dtype)
    angles = synth.uniform_angles(n_angles)
    g = oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=dx, T=T, angles=angles, ndim=ndim, ns=ns, ds=ds)
    G = oracle.forward(g, c, h)
    G = rounded(G + 0.02 * np.mean(G) * rng.standard_normal(G.shape), dtype)
    P = ff.Plan(to_dev(c, dtype), dx, T, angles, ndim=ndim, ns=ns, ds=ds)
    return g, c, h, G, P


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("ds_ratio", [1.0, 0.83, 1.3])
def test_fbp(oracle, dtype, ds_ratio):
    """X^-1 = X^* Lambda; off-grid detector spacings check the filter's scale with
    the multi-bin (0.83 dx) and two-tap (1.3 dx) backprojection."""
    g, c, h, G, P = _case((6, 33, 40), 101, 21, dtype, ds_ratio=ds_ratio)
    with P:
        out = to_np(P.fbp(to_dev(G, dtype)))
    assert rel_l2(out, oracle.fbp(g, G)) <= (1e-12 if dtype == F64 else 2e-6)


@pytest.mark.parametrize("reg", ["l2", "grad"])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_two_step_algorithm9(oracle, dtype, reg):
    g, c, h, G, P = _case((10, 24, 28), 102, 16, dtype)
    flags = oracle.REG_GRAD if reg == "grad" else oracle.POSITIVITY
    lam = 2e-4 if reg == "grad" else 1e-2
    gvol = oracle.fbp(g, G)
    h_ref, obj_ref, s_ref = oracle.fb_two_step(g, c, rounded(gvol, dtype), lam, n_iter=4, n_power=10, flags=flags)
    with P:
        gv = P.fbp(to_dev(G, dtype))
        assert rel_l2(to_np(gv), gvol) <= (1e-12 if dtype == F64 else 2e-6)
        res = P.reconstruct(to_dev(rounded(gvol, dtype), dtype), lam, 4, n_power=10, two_step=True, reg=reg,
                            positivity=(reg == "l2"), cg_tol=1e-14 if dtype == F64 else 0.0)
    tol = TOL_FB[dtype]
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_gradient_regulariser_algorithm8(oracle, dtype):
    g, c, h, G, P = _case((12, 26, 30), 103, 18, dtype)
    lam = 5e-4
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, n_iter=5, n_power=10, flags=oracle.PRECOND | oracle.REG_GRAD)
    with P:
        res = P.reconstruct(to_dev(G, dtype), lam, 5, n_power=10, reg="grad", positivity=False,
                            cg_tol=1e-14 if dtype == F64 else 0.0, cg_maxit=400)
    tol = TOL_FB[dtype]
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", [(12, 26, 30), (8, 20, 70)])
def test_gradient_regulariser_direct_prox(oracle, dtype, shape):
    """Without conjugate-gradient controls a 3D grid solves the prox (I + s lambda N)^-1
    directly by sine transforms along each axis (Sec. 3.2, the prox of R = 1/2 ||D h||^2):
    five FB iterations match the oracle, whose prox is conjugate gradients to 1e-13.
    (8, 20, 70): x lines of 70 points take two k tiles and three j chunks of the
    transform, and no axis has a multiple of 64 columns."""
    nz, ny, nx = shape
    assert nx * nx + ny * ny + nz * nz + nx + ny + nz <= nx * ny * nz     # tables fit: direct solve
    g, c, h, G, P = _case(shape, 107, 18, dtype)
    lam = 5e-4
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, n_iter=5, n_power=10, flags=oracle.PRECOND | oracle.REG_GRAD)
    with P:
        res = P.reconstruct(to_dev(G, dtype), lam, 5, n_power=10, reg="grad", positivity=False)
    tol = TOL_FB[dtype]
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


def test_gradient_regulariser_rejects_positivity():
    import paper_1901_06503_amd as ff
    g, c, h, G, P = _case((4, 10, 12), 104, 5, F64)
    with P:
        with pytest.raises(ff.FfpatError):
            P.reconstruct(to_dev(G, F64), 1e-3, 1, reg="grad", positivity=True)


def test_unknown_reconstruction_flags_are_rejected():
    import ctypes
    from paper_1901_06503_amd import _lib
    g, c, h, G, P = _case((4, 10, 12), 104, 5, F64)
    with P:
        Gd, hd = to_dev(G, F64), to_dev(np.zeros_like(h), F64)
        prm = P._fb_params(Gd, 1e-3, 1, 0.0, 2, True, True, None, None, hd, False, None)
        prm.flags |= 1 << 10
        rc = P._lib.ffpat_reconstruct(P._h, ctypes.c_void_p(Gd.data_ptr()), ctypes.byref(prm),
                                      ctypes.c_void_p(hd.data_ptr()), None, None)
        assert rc == _lib.EINVAL and b"unknown flags" in P._lib.ffpat_last_error()
        assert not hd.any()


@pytest.mark.parametrize("dtype", [F64, F32])
def test_landweber_algorithm7(oracle, dtype):
    g, c, h, G, P = _case((8, 22, 26), 105, 12, dtype)
    h_ref, obj_ref, _ = oracle.fb(g, c, G, 0.0, n_iter=6, n_power=10, flags=oracle.PRECOND)
    with P:
        res = P.landweber(to_dev(G, dtype), 6, n_power=10)
    tol = TOL_FB[dtype]
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)
    assert np.all(np.diff(res.objective) < 0)                 # the data misfit decreases


@pytest.mark.parametrize("dtype", [F64, F32])
def test_landweber_converges_linearly(oracle, dtype):
    """Algorithm 7 is the linear iteration e_{k+1} = (I - s H) e_k for the error e_k
    against the least-squares solution, H = A^T Lambda A (Sec. 3.1).  On a tiny grid
    the dense H comes from the oracle.  H is singular there (few angles), so the
    error is taken on the span of the eigenvectors with eigenvalue >= mu = L / 4,
    where the least-squares solution is unique and H commutes with the projection:
    each GPU iteration shrinks that error by at least rho = max |1 - s lambda| over
    those eigenvalues (about 3/4 with s from the power iteration), and after K
    iterations it equals (I - s H)^K e_0 from the dense spectrum."""
    import paper_1901_06503_amd as ff
    from test_oracle_fb import dense
    g = oracle.Geometry(nx=6, ny=6, nz=4, dx=0.1, T=0.25, angles=synth.uniform_angles(6), ns=8)
    rng = np.random.default_rng(21)
    c = rounded(rng.uniform(0.85, 1.15, size=g.vol_shape), dtype)
    A = dense(lambda f: oracle.forward(g, c, f), g.vol_shape)
    Lam = dense(lambda d: oracle.ramp(g, d), g.data_shape)
    H = A.T @ Lam @ A
    lam, U = np.linalg.eigh(0.5 * (H + H.T))
    G = rounded(rng.normal(size=g.data_shape), dtype)
    b = A.T @ Lam @ G.ravel()
    keep = lam >= 0.25 * lam.max()
    Uk = U[:, keep]
    h_ls = Uk @ ((Uk.T @ b) / lam[keep])          # least squares on the kept span
    K = 24
    with ff.Plan(to_dev(c, dtype), g.dx, g.T, g.angles, ns=g.ns) as P:
        Gd = to_dev(G, dtype)
        h = torch.zeros(P.shape, dtype=dtype, device="cuda")
        s = P.landweber(Gd, 0, n_power=20, h0=h).step     # power iteration only
        errs = [np.linalg.norm(Uk.T @ (to_np(h).ravel() - h_ls))]
        for _ in range(K):
            P.landweber(Gd, 1, h0=h, use_plan_step=True)
            errs.append(np.linalg.norm(Uk.T @ (to_np(h).ravel() - h_ls)))
    rho = np.max(np.abs(1.0 - s * lam[keep]))
    assert 0.5 < rho < 0.9
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    slack = 1e-9 if dtype == F64 else 1e-3
    assert np.all(ratios <= rho + slack)
    pred = np.linalg.norm(((1.0 - s * lam[keep]) ** K) * (Uk.T @ (0.0 - h_ls)))
    assert errs[-1] == pytest.approx(pred, rel=1e-8 if dtype == F64 else 1e-2)
    assert errs[-1] <= rho ** K * errs[0] * (1 + slack)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_limited_data_stripe(oracle, dtype):
    g, c, h, G, P = _case((8, 30, 30), 106, 14, dtype)
    mask = oracle.stripe_mask(g, 0.6)
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G * mask, 1e-3, n_iter=4, n_power=10, det_mask=mask,
                                      flags=oracle.PRECOND | oracle.POSITIVITY)
    with P:
        m = P.stripe_mask(0.6)
        assert np.array_equal(m.cpu().numpy(), mask)
        res = P.reconstruct(to_dev(G * mask, dtype), 1e-3, 4, n_power=10, det_mask=m)
    tol = TOL_FB[dtype]
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol


@pytest.mark.parametrize("dtype", [F64, F32])
def test_two_dimensional_reconstruction(oracle, dtype):
    g, c, h, G, P = _case((1, 48, 48), 107, 30, dtype, ndim=2)
    lam = 1e-3
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, n_iter=5, n_power=10, flags=oracle.PRECOND | oracle.REG_GRAD)
    with P:
        res = P.reconstruct(to_dev(G, dtype), lam, 5, n_power=10, reg="grad", positivity=False,
                            cg_tol=1e-14 if dtype == F64 else 0.0, cg_maxit=400)
    tol = TOL_FB[dtype]
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)

"""Pins of the oracle's Algorithm 8 (Sec. 3.2), its power-iteration step and the
gradient-regulariser prox, on tiny grids where dense linear algebra is exact.

The limits checked here are fixed by the mathematics, not by the oracle:
the normal equations (A^T Lambda A + lambda I) h = A^T Lambda G for the
l2-regularised problem without constraints, the KKT conditions with the
positivity constraint, the largest eigenvalue of A^T Lambda A for the power
iteration, and the closed-form Dirichlet spectrum of the 7-point Laplacian.
"""
import math

import numpy as np
import pytest

from conftest import rel_l2
import synth


def tiny(oracle, n=(6, 6, 4), n_angles=6, ns=8, T=0.25):
    nx, ny, nz = n
    return oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=0.1, T=T, angles=synth.uniform_angles(n_angles), ns=ns)


def dense(apply, in_shape):
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(apply(e.reshape(in_shape))).ravel())
    return np.array(cols).T


@pytest.fixture(scope="module")
def problem(oracle):
    g = tiny(oracle)
    rng = np.random.default_rng(21)
    c = rng.uniform(0.85, 1.15, size=g.vol_shape)
    A = dense(lambda f: oracle.forward(g, c, f), g.vol_shape)
    Lam = dense(lambda d: oracle.ramp(g, d), g.data_shape)
    H = A.T @ Lam @ A
    h_true = np.abs(rng.normal(size=g.vol_shape))
    G = (A @ h_true.ravel()).reshape(g.data_shape) + 0.05 * rng.normal(size=g.data_shape)
    return dict(g=g, c=c, A=A, Lam=Lam, H=0.5 * (H + H.T), G=G)


def test_dense_adjoint_equals_transpose(oracle, problem):
    g, c, A = problem["g"], problem["c"], problem["A"]
    AT = dense(lambda d: oracle.adjoint(g, c, d), g.data_shape)
    assert np.max(np.abs(AT - A.T)) <= 1e-12 * np.max(np.abs(A))


def test_power_iteration_converges_to_top_eigenvalue(oracle, problem):
    g, c, H = problem["g"], problem["c"], problem["H"]
    lam_max = np.linalg.eigvalsh(H).max()
    L20, hist = oracle.power(g, c, 20)
    assert np.all(np.diff(hist) >= -1e-12 * lam_max)     # Rayleigh-type estimate increases
    assert L20 <= lam_max * (1 + 1e-12)
    L_long, _ = oracle.power(g, c, 1500)
    assert L_long == pytest.approx(lam_max, rel=1e-10)


def test_fb_without_constraint_converges_to_normal_equations(oracle, problem):
    g, c, H, A, Lam, G = (problem[k] for k in ("g", "c", "H", "A", "Lam", "G"))
    lam_max = np.linalg.eigvalsh(H).max()
    lam = 0.3 * lam_max
    s = 1.0 / lam_max
    ref = np.linalg.solve(H + lam * np.eye(H.shape[0]), A.T @ Lam @ G.ravel())
    h, obj, s_used = oracle.fb(g, c, G, lam, step=s, n_iter=400, flags=oracle.PRECOND)
    assert s_used == s
    assert rel_l2(h.ravel(), ref) <= 1e-10
    assert np.all(np.diff(obj) <= 1e-12 * abs(obj[0]))   # FB with s <= 1/L decreases the objective


def test_landweber_converges_linearly_on_the_well_conditioned_span(oracle, problem):
    """Algorithm 7 (Sec. 3.1) without regulariser or constraint is the linear iteration
    e_{k+1} = (I - s H) e_k, H = A^T Lambda A.  On the span of the eigenvectors with
    eigenvalue >= L / 4 (H is singular on this grid) the error shrinks every step by
    at least rho = max |1 - s lambda| there, and equals (I - s H)^k e_0."""
    g, c, H, A, Lam, G = (problem[k] for k in ("g", "c", "H", "A", "Lam", "G"))
    lam, U = np.linalg.eigh(H)
    keep = lam >= 0.25 * lam.max()
    Uk = U[:, keep]
    b = A.T @ Lam @ G.ravel()
    h_ls = Uk @ ((Uk.T @ b) / lam[keep])
    _, _, s = oracle.fb(g, c, G, 0.0, step=0.0, n_iter=0, n_power=20, flags=oracle.PRECOND)
    errs = []
    for k in range(0, 21, 4):
        h, _, _ = oracle.fb(g, c, G, 0.0, step=s, n_iter=k, flags=oracle.PRECOND)
        errs.append(np.linalg.norm(Uk.T @ (h.ravel() - h_ls)))
    rho = np.max(np.abs(1.0 - s * lam[keep]))
    assert 0.5 < rho < 0.9
    assert np.all(np.array(errs[1:]) <= rho ** 4 * np.array(errs[:-1]) * (1 + 1e-10))
    pred = np.linalg.norm(((1.0 - s * lam[keep]) ** 20) * (Uk.T @ h_ls))
    assert errs[-1] == pytest.approx(pred, rel=1e-9)


def test_fb_with_positivity_satisfies_kkt(oracle, problem):
    g, c, H, A, Lam, G = (problem[k] for k in ("g", "c", "H", "A", "Lam", "G"))
    lam_max = np.linalg.eigvalsh(H).max()
    lam = 0.3 * lam_max
    h, obj, _ = oracle.fb(g, c, G, lam, step=1.0 / lam_max, n_iter=600,
                          flags=oracle.PRECOND | oracle.POSITIVITY)
    h = h.ravel()
    grad = H @ h - A.T @ Lam @ G.ravel() + lam * h
    scale = np.max(np.abs(A.T @ Lam @ G.ravel()))
    assert h.min() >= 0
    pos = h > 1e-12 * np.max(h)
    assert np.max(np.abs(grad[pos])) <= 1e-8 * scale
    assert grad[~pos].min() >= -1e-8 * scale
    assert (~pos).sum() > 0                               # the constraint is active somewhere


def test_fb_without_precond_uses_plain_least_squares(oracle, problem):
    g, c, A, G = (problem[k] for k in ("g", "c", "A", "G"))
    H = A.T @ A
    lam_max = np.linalg.eigvalsh(H).max()
    lam = 0.3 * lam_max
    ref = np.linalg.solve(H + lam * np.eye(H.shape[0]), A.T @ G.ravel())
    h, _, _ = oracle.fb(g, c, G, lam, step=1.0 / lam_max, n_iter=400, flags=0)
    assert rel_l2(h.ravel(), ref) <= 1e-10


def test_fb_objective_at_exact_solution(oracle, problem):
    # with noise-free data and h0 = h_true the residual vanishes: J_0 = lambda/2 ||h_true||^2
    g, c, A = problem["g"], problem["c"], problem["A"]
    h_true = synth.random_field(g.vol_shape, 22)
    G = (A @ h_true.ravel()).reshape(g.data_shape)
    _, obj, _ = oracle.fb(g, c, G, 0.7, step=1e-3, n_iter=1, flags=oracle.PRECOND, h0=h_true)
    assert obj[0] == pytest.approx(0.35 * np.sum(h_true ** 2), rel=1e-10)


def test_fb_detector_mask_equals_masked_least_squares(oracle, problem):
    g, c, A, Lam, G = (problem[k] for k in ("g", "c", "A", "Lam", "G"))
    mask = np.ones(g.data_shape, dtype=np.uint8)
    mask[:, :, 3:5] = 0                                  # a missing central stripe of bins
    M = np.diag(mask.ravel().astype(np.float64))
    H = A.T @ M @ Lam @ M @ A
    H = 0.5 * (H + H.T)
    lam_max = np.linalg.eigvalsh(H).max()
    lam = 0.3 * lam_max
    ref = np.linalg.solve(H + lam * np.eye(H.shape[0]), A.T @ M @ Lam @ M @ G.ravel())
    h, _, _ = oracle.fb(g, c, G, lam, step=1.0 / lam_max, n_iter=400, flags=oracle.PRECOND, det_mask=mask)
    assert rel_l2(h.ravel(), ref) <= 1e-10
    L, _ = oracle.power(g, c, 1500, det_mask=mask)
    assert L == pytest.approx(lam_max, rel=1e-8)


def test_fb_support_mask_zeroes_outside(oracle, problem):
    g, c, G = problem["g"], problem["c"], problem["G"]
    sup = np.zeros(g.vol_shape, dtype=np.uint8)
    sup[1:3, 2:5, 1:5] = 1
    h, _, _ = oracle.fb(g, c, G, 1e-3, n_iter=3, support=sup)
    assert np.all(h[sup == 0] == 0.0)
    assert np.any(h[sup == 1] != 0.0)


# ---------------------------------------------------------------- gradient regulariser
def test_neg_lap7_dirichlet_spectrum(oracle):
    g = oracle.Geometry(nx=5, ny=4, nz=3, dx=0.2, T=0.1, angles=synth.uniform_angles(2))
    M = dense(lambda f: oracle.neg_lap7(g, f), g.vol_shape)
    assert np.max(np.abs(M - M.T)) == 0.0
    ev = np.sort(np.linalg.eigvalsh(M))
    one = lambda n: (2 - 2 * np.cos(np.arange(1, n + 1) * math.pi / (n + 1))) / g.dx ** 2
    ref = np.sort((one(5)[None, None, :] + one(4)[None, :, None] + one(3)[:, None, None]).ravel())
    assert np.max(np.abs(ev - ref)) <= 1e-11 * ref.max()


def test_prox_grad_solves_its_equation(oracle):
    g = oracle.Geometry(nx=9, ny=8, nz=7, dx=0.1, T=0.1, angles=synth.uniform_angles(2))
    f = synth.random_field(g.vol_shape, 23)
    tau = 0.01
    h = oracle.prox_grad(g, tau, f)
    res = h + tau * oracle.neg_lap7(g, h) - f
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(f)
    # prox minimises 1/2||h - f||^2 + tau/2 ||D h||^2: compare against random perturbations
    def F(u):
        return 0.5 * np.sum((u - f) ** 2) + 0.5 * tau * np.sum(u * oracle.neg_lap7(g, u))
    rng = np.random.default_rng(0)
    for _ in range(5):
        assert F(h) < F(h + 1e-3 * rng.normal(size=h.shape))


def test_fb_gradient_regulariser_converges_to_normal_equations(oracle, problem):
    g, c, H, A, Lam, G = (problem[k] for k in ("g", "c", "H", "A", "Lam", "G"))
    D = dense(lambda f: oracle.neg_lap7(g, f), g.vol_shape)
    lam_max = np.linalg.eigvalsh(H).max()
    lam = 0.05 * lam_max * g.dx ** 2
    ref = np.linalg.solve(H + lam * D, A.T @ Lam @ G.ravel())
    h, _, _ = oracle.fb(g, c, G, lam, step=1.0 / lam_max, n_iter=2000, flags=oracle.PRECOND | oracle.REG_GRAD)
    assert rel_l2(h.ravel(), ref) <= 1e-8


# ---------------------------------------------------------------- two-step method (Algorithm 9)
def test_fbp_inverts_the_xray_transform_on_smooth_objects(oracle):
    """X^-1 = X^* Lambda (Sec. 3.1): fbp(X v) ~ v."""
    n = 64
    dx = synth.grid_spacing(n)
    g = oracle.Geometry(nx=n, ny=n, nz=2, dx=dx, T=0.1, angles=synth.uniform_angles(96))
    vol = synth.gaussian_blob(g.vol_shape, dx, (-0.15, 0.2, 0.0), 4 * dx)
    rec = oracle.fbp(g, oracle.project(g, vol))
    inner = np.hypot(*np.meshgrid(synth.axis(n, dx), synth.axis(n, dx))) < 1.0
    for z in range(2):
        assert rel_l2(rec[z][inner], vol[z][inner]) < 0.05


@pytest.mark.parametrize("ratio", [0.83, 1.3])
def test_fbp_inverts_with_off_grid_detector_spacing(oracle, ratio):
    """X^-1 = X^* Lambda with detector bins ds = ratio * dx (0.83: footprints wider
    than one bin, several taps per voxel; 1.3: at most two); the scale of the
    inverse does not depend on ds."""
    n = 64
    dx = synth.grid_spacing(n)
    ds = ratio * dx
    ns = int(math.ceil(n * dx / ds)) + 8
    g = oracle.Geometry(nx=n, ny=n, nz=2, dx=dx, T=0.1, angles=synth.uniform_angles(96), ns=ns, ds=ds)
    vol = synth.gaussian_blob(g.vol_shape, dx, (-0.15, 0.2, 0.0), 4 * dx)
    rec = oracle.fbp(g, oracle.project(g, vol))
    inner = np.hypot(*np.meshgrid(synth.axis(n, dx), synth.axis(n, dx))) < 1.0
    for z in range(2):
        r, v = rec[z][inner], vol[z][inner]
        assert np.vdot(r, v) / np.vdot(r, r) == pytest.approx(1.0, abs=0.02)
        assert rel_l2(r, v) < 0.08


@pytest.fixture(scope="module")
def wave_problem(oracle):
    g = tiny(oracle, n=(5, 5, 4))
    rng = np.random.default_rng(31)
    c = rng.uniform(0.85, 1.15, size=g.vol_shape)
    W = dense(lambda f: oracle.wave(g, c, f), g.vol_shape)
    gv = rng.normal(size=g.vol_shape)
    return g, c, W, gv


def test_two_step_fb_converges_to_normal_equations(oracle, wave_problem):
    g, c, W, gv = wave_problem
    H = W.T @ W
    lam_max = np.linalg.eigvalsh(0.5 * (H + H.T)).max()
    lam = 0.3 * lam_max
    ref = np.linalg.solve(H + lam * np.eye(H.shape[0]), W.T @ gv.ravel())
    h, obj, s = oracle.fb_two_step(g, c, gv, lam, step=1.0 / lam_max, n_iter=300, flags=0)
    assert rel_l2(h.ravel(), ref) <= 1e-10
    assert np.all(np.diff(obj) <= 1e-12 * abs(obj[0]))
    _, _, s_pow = oracle.fb_two_step(g, c, gv, lam, step=0.0, n_iter=0, n_power=3000, flags=0)
    assert 1.0 / s_pow == pytest.approx(lam_max, rel=1e-10)


def test_two_step_fb_gradient_regulariser(oracle, wave_problem):
    g, c, W, gv = wave_problem
    H = W.T @ W
    D = dense(lambda f: oracle.neg_lap7(g, f), g.vol_shape)
    lam_max = np.linalg.eigvalsh(0.5 * (H + H.T)).max()
    lam = 0.02 * lam_max * g.dx ** 2
    ref = np.linalg.solve(H + lam * D, W.T @ gv.ravel())
    h, _, _ = oracle.fb_two_step(g, c, gv, lam, step=1.0 / lam_max, n_iter=1500, flags=oracle.REG_GRAD)
    assert rel_l2(h.ravel(), ref) <= 1e-8


def test_stripe_mask(oracle):
    g = oracle.Geometry(nx=11, ny=11, nz=2, dx=0.2, T=0.1, angles=synth.uniform_angles(3))
    m = oracle.stripe_mask(g, 0.5)
    assert m.shape == g.data_shape
    s = (np.arange(11) - 5) * 0.2
    assert np.array_equal(m[1, 1], (np.abs(s) > 0.5).astype(np.uint8))

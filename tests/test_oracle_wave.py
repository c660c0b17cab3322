"""Pins of the oracle's wave operator W_T and its transpose (CPU only).

The oracle's Laplacian, leapfrog and transpose are checked against facts
that do not come from the oracle itself: polynomial exactness of the
fourth-order stencil, symmetry and definiteness, the Chebyshev closed form of
the two-level recursion, conservation of the scheme's discrete energy, the
constant-speed radial solution of the 3D wave equation (Sec. 2.1, eq.
wave1/wave2 with zero initial velocity), and the adjoint identity.
"""
import math

import numpy as np
import pytest

from conftest import rel_l2
import synth


def geom(oracle, nx, ny, nz, dx=0.1, T=0.3, n_angles=4, cfl=0.3, ndim=3):
    return oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=dx, T=T, angles=synth.uniform_angles(n_angles),
                           cfl=cfl, ndim=ndim)


def dense_operator(apply, shape):
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, i] = apply(e.reshape(shape)).ravel()
    return M


# ---------------------------------------------------------------- time grid
def test_time_grid_hits_T_and_respects_cfl(oracle):
    for N, cmax in [(48, 1.15), (128, 1.2), (256, 1.2), (384, 1.25), (64, 1.2), (192, 1.2)]:
        dx = synth.grid_spacing(N)
        nt, dt = oracle.time_grid(0.5, cmax, 0.3, dx)
        assert nt * dt == pytest.approx(0.5, rel=1e-15)
        assert cmax * dt / dx <= 0.3 * (1 + 1e-12)       # never coarser than the CFL target
        assert cmax * (0.5 / (nt - 1)) / dx > 0.3         # and one step fewer would break it


def test_time_grid_exact_tie_is_not_rounded_up(oracle):
    # T c_max / (cfl dx) = 170 exactly (up to rounding) at 256^3, c_max = 1.2
    nt, _ = oracle.time_grid(0.5, 1.2, 0.3, synth.grid_spacing(256))
    assert nt == 170
    nt, _ = oracle.time_grid(0.5, 1.2, 0.3, synth.grid_spacing(64))
    assert nt == 42


# ---------------------------------------------------------------- Laplacian
def test_laplacian_exact_on_quintic_polynomials(oracle):
    n = 14
    dx = 0.07
    g = geom(oracle, n, n, n, dx=dx)
    ax = synth.axis(n, dx)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    rng = np.random.default_rng(0)
    # random polynomial of total degree <= 5 and its exact Laplacian
    f = np.zeros_like(X)
    lap = np.zeros_like(X)
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                co = rng.normal()
                f += co * X ** a * Y ** b * Z ** c
                if a >= 2:
                    lap += co * a * (a - 1) * X ** (a - 2) * Y ** b * Z ** c
                if b >= 2:
                    lap += co * b * (b - 1) * X ** a * Y ** (b - 2) * Z ** c
                if c >= 2:
                    lap += co * c * (c - 1) * X ** a * Y ** b * Z ** (c - 2)
    out = oracle.laplacian(g, f)
    inner = (slice(2, -2),) * 3
    assert np.max(np.abs(out[inner] - lap[inner])) <= 1e-9 * np.max(np.abs(lap[inner]))


def test_laplacian_symmetric_negative_definite_with_bound(oracle):
    g = geom(oracle, 7, 5, 6, dx=0.2)
    L = dense_operator(lambda f: oracle.laplacian(g, f), g.vol_shape)
    assert np.max(np.abs(L - L.T)) <= 1e-12 * np.max(np.abs(L))
    ev = np.linalg.eigvalsh(0.5 * (L + L.T))
    assert ev.max() < 0
    # symbol of the 1D stencil ranges over (-16/3, 0] / dx^2 per axis
    assert ev.min() > -3 * 16.0 / 3.0 / g.dx ** 2


def test_laplacian_zero_ghosts_at_corner(oracle):
    # a unit impulse at a corner spreads exactly to the in-grid stencil points;
    # symmetry pins the boundary rule (mirror or clamp ghosts would break it)
    g = geom(oracle, 6, 6, 6, dx=1.0)
    rng = np.random.default_rng(1)
    u = rng.normal(size=g.vol_shape)
    v = rng.normal(size=g.vol_shape)
    lhs = np.vdot(oracle.laplacian(g, u), v)
    rhs = np.vdot(u, oracle.laplacian(g, v))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_laplacian_2d_mode_ignores_z(oracle):
    g3 = geom(oracle, 9, 8, 5)
    g2 = geom(oracle, 9, 8, 5, ndim=2)
    f = synth.random_field(g3.vol_shape, 3)
    out2 = oracle.laplacian(g2, f)
    for z in range(5):
        single = geom(oracle, 9, 8, 1, ndim=2)
        assert np.allclose(out2[z], oracle.laplacian(single, f[z:z + 1])[0], rtol=0, atol=1e-12)
    assert not np.allclose(out2, oracle.laplacian(g3, f))


# ---------------------------------------------------------------- W_T
def _kappa(oracle, g, c):
    nt, dt, _ = oracle.plan_info(g, c)
    return nt, (c * dt) ** 2


def test_wave_matches_chebyshev_closed_form(oracle):
    """p(n) = T_n(I + K L / 2) h: evaluate T_n through the eigendecomposition of
    the symmetric matrix K^{1/2} L K^{1/2} and cos(n arccos(1 + mu/2))."""
    g = geom(oracle, 6, 5, 4, dx=0.1, T=0.45)
    rng = np.random.default_rng(2)
    c = rng.uniform(0.8, 1.2, size=g.vol_shape)
    h = rng.normal(size=g.vol_shape)
    nt, kappa = _kappa(oracle, g, c)
    assert nt >= 10
    L = dense_operator(lambda f: oracle.laplacian(g, f), g.vol_shape)
    d = np.sqrt(kappa.ravel())
    S = d[:, None] * L * d[None, :]
    mu, U = np.linalg.eigh(0.5 * (S + S.T))
    x = 1.0 + 0.5 * mu
    assert np.all(x >= -1) and np.all(x <= 1)
    Tn = np.cos(nt * np.arccos(x))
    ref = d * (U @ (Tn * (U.T @ (h.ravel() / d))))
    out = oracle.wave(g, c, h)
    assert rel_l2(out.ravel(), ref) <= 1e-12


def test_wave_single_step_is_symmetric_start(oracle):
    # with n_t = 1 (T tiny) W_T = I + K L / 2: zero initial velocity (eq. wave2)
    g = geom(oracle, 7, 6, 5, dx=0.1, T=0.01)
    rng = np.random.default_rng(4)
    c = rng.uniform(0.9, 1.1, size=g.vol_shape)
    h = rng.normal(size=g.vol_shape)
    nt, kappa = _kappa(oracle, g, c)
    assert nt == 1
    L = dense_operator(lambda f: oracle.laplacian(g, f), g.vol_shape)
    ref = h.ravel() + 0.5 * kappa.ravel() * (L @ h.ravel())
    assert rel_l2(oracle.wave(g, c, h).ravel(), ref) <= 1e-14


def test_leapfrog_discrete_energy_is_conserved(oracle):
    g = geom(oracle, 16, 14, 12, dx=0.1, T=1.0)
    rng = np.random.default_rng(5)
    c = rng.uniform(0.8, 1.2, size=g.vol_shape)
    h = rng.normal(size=g.vol_shape)
    hist = oracle.wave_history(g, c, h, 40)
    E = [oracle.energy(g, c, hist[k], hist[k + 1]) for k in range(40)]
    E = np.array(E)
    assert np.max(np.abs(E - E[0])) <= 1e-12 * abs(E[0])
    assert E[0] > 0


def test_wave_time_reversal(oracle):
    # the leapfrog is time-symmetric: stepping back from (p(n), p(n-1)) returns h
    g = geom(oracle, 10, 9, 8, dx=0.1, T=1.0)
    rng = np.random.default_rng(6)
    c = rng.uniform(0.8, 1.2, size=g.vol_shape)
    h = rng.normal(size=g.vol_shape)
    nt, kappa = _kappa(oracle, g, c)
    hist = oracle.wave_history(g, c, h, nt)
    cur, prev = hist[nt - 1], hist[nt]      # reversed order
    for _ in range(nt - 1):
        cur, prev = 2 * cur - prev + kappa * oracle.laplacian(g, cur), cur
    assert rel_l2(cur, h) <= 1e-10


def _radial_reference(r, t, c0, sigma):
    """p(r,t) for p(.,0) = f(|r|), f = Gaussian, dp/dt(.,0) = 0, speed c0 in R^3."""
    f = lambda u: np.exp(-u * u / (2 * sigma * sigma))
    fp = lambda u: -u / (sigma * sigma) * f(u)
    ct = c0 * t
    with np.errstate(invalid="ignore", divide="ignore"):
        p = ((r - ct) * f(r - ct) + (r + ct) * f(r + ct)) / (2 * r)
    p0 = f(ct) + ct * fp(ct)
    return np.where(r > 1e-12, p, p0)


@pytest.mark.slow
def test_wave_constant_speed_radial_closed_form_second_order(oracle):
    sigma, T, c0 = 0.15, 0.5, 1.0
    errs = []
    for n in (61, 121):
        dx = 3.0 / (n - 1)
        g = geom(oracle, n, n, n, dx=dx, T=T)
        ax = synth.axis(n, dx)
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        r = np.sqrt(X * X + Y * Y + Z * Z)
        h = np.exp(-r * r / (2 * sigma * sigma))
        c = np.full(g.vol_shape, c0)
        p = oracle.wave(g, c, h)
        errs.append(rel_l2(p, _radial_reference(r, T, c0, sigma)))
    assert errs[1] < 2e-3
    assert errs[0] / errs[1] > 3.0      # order ~2 under refinement at fixed cfl


# ---------------------------------------------------------------- W_T^T
def test_wave_transpose_dot_test(oracle):
    g = geom(oracle, 13, 11, 9, dx=0.1, T=0.8)
    rng = np.random.default_rng(7)
    c = rng.uniform(0.8, 1.2, size=g.vol_shape)
    h = rng.normal(size=g.vol_shape)
    q = rng.normal(size=g.vol_shape)
    lhs = np.vdot(oracle.wave(g, c, h), q)
    rhs = np.vdot(h, oracle.wave_T(g, c, q))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(h) * np.linalg.norm(q) * 10


def test_wave_transpose_dense_and_conjugation(oracle):
    g = geom(oracle, 5, 5, 4, dx=0.1, T=0.5)
    rng = np.random.default_rng(8)
    c = rng.uniform(0.8, 1.2, size=g.vol_shape)
    W = dense_operator(lambda f: oracle.wave(g, c, f), g.vol_shape)
    WT = dense_operator(lambda f: oracle.wave_T(g, c, f), g.vol_shape)
    assert np.max(np.abs(WT - W.T)) <= 1e-12 * np.max(np.abs(W))
    # W^T = K^{-1} W K (the scheme is a polynomial in K L)
    _, kappa = _kappa(oracle, g, c)
    q = rng.normal(size=g.vol_shape)
    alt = oracle.wave(g, c, kappa * q) / kappa
    assert rel_l2(alt, oracle.wave_T(g, c, q)) <= 1e-12


def test_wave_is_identity_plus_kL_for_constant_field_in_interior(oracle):
    # a constant field away from the boundary does not evolve in the interior (L 1 = 0 inside)
    g = geom(oracle, 20, 20, 20, dx=0.1, T=0.05)
    c = np.ones(g.vol_shape)
    h = np.ones(g.vol_shape)
    nt, _ = _kappa(oracle, g, c)
    p = oracle.wave(g, c, h)
    m = 2 * nt + 2
    inner = (slice(m, -m),) * 3
    assert np.max(np.abs(p[inner] - 1.0)) <= 1e-12

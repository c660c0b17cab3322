"""Pins of the oracle's X-ray transform X, its transpose and the ramp filter Lambda.

Checked against: a brute-force ray march written here from the definition of
the X-ray transform with linear interpolation (eq. Radon, Sec. 4.1), the
closed-form projection of a Gaussian, plane-by-plane action (Sec. 2.1), the
adjoint identity, the Ram-Lak symbol |omega|/(2 pi), positive definiteness,
the filtered-backprojection identity X^* Lambda = X^{-1} (Sec. 3.1), and the
1D d'Alembert law for plane integrals of a constant-speed wave (Sec. 2.2).
"""
import math

import numpy as np
import pytest

from conftest import rel_l2
import synth


def geom(oracle, nx, ny, nz, dx=0.1, n_angles=8, ns=0, ds=0.0, T=0.3, angles=None):
    if angles is None:
        angles = synth.uniform_angles(n_angles)
    return oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=dx, T=T, angles=angles, ns=ns, ds=ds)


def brute_force_ray_march(vol, dx, angles, ns, ds):
    """For each angle and bin: walk the ray {x cos a + y sin a = s} one grid line
    of the major axis at a time, interpolate linearly along the minor axis
    (zero outside the grid) and multiply the sum by the step length dx / m."""
    nz, ny, nx = vol.shape
    xs = (np.arange(nx) - 0.5 * (nx - 1)) * dx
    ys = (np.arange(ny) - 0.5 * (ny - 1)) * dx
    out = np.zeros((len(angles), nz, ns))

    def lerp(line, pos):  # pos in index units along the line
        i0 = math.floor(pos)
        f = pos - i0
        v0 = line[i0] if 0 <= i0 < len(line) else 0.0
        v1 = line[i0 + 1] if 0 <= i0 + 1 < len(line) else 0.0
        return (1 - f) * v0 + f * v1

    for a, phi in enumerate(angles):
        ca, sa = math.cos(phi), math.sin(phi)
        for j in range(ns):
            s = (j - 0.5 * (ns - 1)) * ds
            for z in range(nz):
                acc = 0.0
                if abs(ca) >= abs(sa):       # ray runs mostly along y: step over rows
                    for k in range(ny):
                        xstar = (s - ys[k] * sa) / ca
                        acc += lerp(vol[z, k, :], (xstar - xs[0]) / dx)
                    acc *= dx / abs(ca)
                else:                         # ray runs mostly along x: step over columns
                    for i in range(nx):
                        ystar = (s - xs[i] * ca) / sa
                        acc += lerp(vol[z, :, i], (ystar - ys[0]) / dx)
                    acc *= dx / abs(sa)
                out[a, z, j] = acc
    return out


def test_project_equals_brute_force_ray_march(oracle):
    angles = np.array([0.0, 0.3, math.pi / 4, 1.2, math.pi / 2, 2.0, 3 * math.pi / 4, 2.9])
    for (nx, ny, ns, ds) in [(8, 7, 9, 0.1), (9, 10, 12, 0.07)]:
        g = geom(oracle, nx, ny, 3, dx=0.1, ns=ns, ds=ds, angles=angles)
        vol = synth.random_field(g.vol_shape, 11)
        ref = brute_force_ray_march(vol, g.dx, angles, ns, ds)
        assert np.max(np.abs(oracle.project(g, vol) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_project_gaussian_closed_form(oracle):
    n, sig = 64, 3.2
    dx = synth.grid_spacing(n)
    sigma = sig * dx
    x0 = (0.21, -0.13, 0.05)
    angles = np.array([0.0, 0.4, math.pi / 4, 1.3, math.pi / 2, 2.2, 2.8])
    g = geom(oracle, n, n, n, dx=dx, angles=angles)
    vol = synth.gaussian_blob(g.vol_shape, dx, x0, sigma, amplitude=1.7)
    out = oracle.project(g, vol)
    s = synth.axis(n, dx)
    z = synth.axis(n, dx)
    for a, phi in enumerate(angles):
        t0 = x0[0] * math.cos(phi) + x0[1] * math.sin(phi)
        ref = 1.7 * math.sqrt(2 * math.pi) * sigma * np.exp(
            -((s[None, :] - t0) ** 2 + (z[:, None] - x0[2]) ** 2) / (2 * sigma ** 2))
        assert rel_l2(out[a], ref) < 1e-2


def test_project_acts_plane_by_plane(oracle):
    g = geom(oracle, 12, 11, 6, dx=0.1, ns=14)
    vol = np.zeros(g.vol_shape)
    vol[3] = synth.random_field(g.vol_shape[1:], 12)
    out = oracle.project(g, vol)
    assert np.all(out[:, [0, 1, 2, 4, 5], :] == 0.0)
    g1 = geom(oracle, 12, 11, 1, dx=0.1, ns=14)
    assert np.max(np.abs(out[:, 3, :] - oracle.project(g1, vol[3:4])[:, 0, :])) <= 1e-14


def test_backproject_is_transpose(oracle):
    g = geom(oracle, 13, 12, 5, dx=0.1, n_angles=17, ns=15, ds=0.09)
    rng = np.random.default_rng(13)
    v = rng.normal(size=g.vol_shape)
    d = rng.normal(size=g.data_shape)
    lhs = np.vdot(oracle.project(g, v), d)
    rhs = np.vdot(v, oracle.backproject(g, d))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(v) * np.linalg.norm(d))


# ---------------------------------------------------------------- Lambda
def test_ramlak_symbol_is_abs_omega_over_2pi(oracle):
    taps = np.array([oracle.ramlak_tap(k) for k in range(0, 4001)])
    assert taps[0] == 0.25 and taps[2] == 0.0 and taps[1] == pytest.approx(-1 / math.pi ** 2)
    n = np.arange(1, 200001, 2, dtype=np.float64)
    for w in [0.0, 0.3, 1.0, 2.0, 3.0]:
        H = 0.25 - 2.0 / math.pi ** 2 * np.sum(np.cos(n * w) / n ** 2)
        assert H == pytest.approx(abs(w) / (2 * math.pi), abs=1e-5)


def test_ramp_symmetric_positive_definite(oracle):
    g = geom(oracle, 4, 4, 1, dx=0.1, n_angles=1, ns=64)
    cols = []
    for j in range(64):
        e = np.zeros(g.data_shape)
        e[0, 0, j] = 1.0
        cols.append(oracle.ramp(g, e)[0, 0])
    M = np.array(cols).T
    assert np.max(np.abs(M - M.T)) == 0.0
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > 0
    # Toeplitz: constant along diagonals
    assert np.allclose(np.diag(M, 1), M[0, 1]) and np.allclose(np.diag(M, 3), M[0, 3])
    assert np.all(np.diag(M, 2) == 0.0)


def test_fbp_identity_backproject_ramp_project(oracle):
    """X^T Lambda X ~ I on a smooth object (filtered backprojection, Sec. 3.1)."""
    n = 64
    dx = synth.grid_spacing(n)
    g = geom(oracle, n, n, 1, dx=dx, n_angles=96)
    vol = synth.gaussian_blob((1, n, n), dx, (0.2, -0.1, 0.0), 4 * dx)
    rec = oracle.backproject(g, oracle.ramp(g, oracle.project(g, vol)))
    inner = np.hypot(*np.meshgrid(synth.axis(n, dx), synth.axis(n, dx))) < 1.0
    assert rel_l2(rec[0][inner], vol[0][inner]) < 0.05


@pytest.mark.parametrize("ratio,tol", [(0.6, 0.05), (0.83, 0.05), (1.3, 0.08), (2.0, 0.2)])
def test_fbp_identity_off_grid_detector_spacing(oracle, ratio, tol):
    """X^T Lambda X ~ I (Sec. 3.1) with detector bins ds = ratio * dx.  X's ray sums do
    not depend on ds, X^T spreads each bin over a footprint of dx^2 / ds in bins, and
    the Ram-Lak sum over bins approximates ds times the ramp filter: the ds factors
    cancel and the scale of Lambda is pi / (N_angles dx^2) for any ds.  The best scalar
    fit of the reconstruction to the object is 1 within 2% at every ratio; a scale with
    ds dx or ds^2 in place of dx^2 would miss it by the factor ds/dx or (ds/dx)^2
    (0.6 .. 4).  Coarse detectors (ds > m dx) sample the footprint unevenly, so the
    residual ripple grows with the ratio."""
    n = 64
    dx = synth.grid_spacing(n)
    ds = ratio * dx
    ns = int(math.ceil(n * dx / ds)) + 8
    g = geom(oracle, n, n, 1, dx=dx, n_angles=96, ns=ns, ds=ds)
    vol = synth.gaussian_blob((1, n, n), dx, (0.2, -0.1, 0.0), 4 * dx)
    rec = oracle.backproject(g, oracle.ramp(g, oracle.project(g, vol)))
    inner = np.hypot(*np.meshgrid(synth.axis(n, dx), synth.axis(n, dx))) < 1.0
    r, v = rec[0][inner], vol[0][inner]
    assert np.vdot(r, v) / np.vdot(r, r) == pytest.approx(1.0, abs=0.02)
    assert rel_l2(r, v) < tol


# ---------------------------------------------------------------- X and W together
@pytest.mark.slow
def test_plane_integrals_follow_dalembert(oracle):
    """Constant speed: integrating the projections over z gives plane integrals
    R p(phi, s, T) = 1/2 (R h(phi, s - cT) + R h(phi, s + cT)) (Sec. 2.2)."""
    n = 81
    dx = synth.grid_spacing(n)
    k_shift = 16
    T = k_shift * dx           # c = 1: shift by exactly 16 bins
    angles = np.array([0.0, 0.5, math.pi / 4, 2.0])
    g = geom(oracle, n, n, n, dx=dx, angles=angles, T=T)
    h = synth.gaussian_blob(g.vol_shape, dx, (0.1, 0.05, -0.05), 3 * dx)
    c = np.ones(g.vol_shape)
    Rh = oracle.project(g, h).sum(axis=1) * dx
    Rp = oracle.forward(g, c, h).sum(axis=1) * dx
    ref = np.zeros_like(Rh)
    ref[:, k_shift:] += 0.5 * Rh[:, :-k_shift]
    ref[:, :-k_shift] += 0.5 * Rh[:, k_shift:]
    assert rel_l2(Rp, ref) < 2e-2

"""Property pins of the oracle over random small geometries (hypothesis, derandomized).

Each property is a fact the definitions fix, checked on many shapes, angle sets,
detector spacings and sound speeds rather than on one hand-picked case:
  * X equals a brute-force ray march written from eq. Radon (linear interpolation
    along the minor axis, Sec. 4.1), for any angle, bin count and spacing;
  * <X v, g> = <v, X^T g> (X^T is the transpose of X);
  * <W_T h, g> = <h, W_T^T g> for any speed inside the stability bound and any n_t;
  * Lambda is symmetric and positive definite for any row length;
  * with positivity, every Algorithm-8 iterate is non-negative and the objective
    never increases (s <= 1/L with L the top eigenvalue from a long power iteration).
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from conftest import rel_l2
from test_oracle_xray import brute_force_ray_march

SETTINGS = dict(max_examples=15, deadline=None, derandomize=True)


def _geom(oracle, nx, ny, nz, angles, ns=0, ds_ratio=1.0, dx=0.1, T=0.3):
    return oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=dx, T=T, angles=np.asarray(angles, dtype=np.float64),
                           ns=ns, ds=ds_ratio * dx)


angle_sets = st.lists(st.floats(min_value=0.0, max_value=math.pi, allow_nan=False, exclude_max=True),
                      min_size=1, max_size=4)


@settings(**SETTINGS)
@given(nx=st.integers(2, 8), ny=st.integers(2, 8), nz=st.integers(1, 2), angles=angle_sets,
       ns_extra=st.integers(-1, 3), ds_ratio=st.sampled_from([0.6, 1.0, 1.4]), seed=st.integers(0, 2 ** 16))
def test_project_equals_ray_march_on_random_geometries(oracle, nx, ny, nz, angles, ns_extra, ds_ratio, seed):
    ns = max(1, nx + ns_extra)
    g = _geom(oracle, nx, ny, nz, angles, ns=ns, ds_ratio=ds_ratio)
    v = np.random.default_rng(seed).standard_normal((nz, ny, nx))
    ref = brute_force_ray_march(v, g.dx, g.angles, ns, g.ds)
    got = oracle.project(g, v)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


@settings(**SETTINGS)
@given(nx=st.integers(2, 12), ny=st.integers(2, 12), nz=st.integers(1, 3), angles=angle_sets,
       ns_extra=st.integers(-2, 4), ds_ratio=st.sampled_from([0.5, 0.83, 1.0, 1.3, 2.0]),
       seed=st.integers(0, 2 ** 16))
def test_backproject_is_the_transpose_on_random_geometries(oracle, nx, ny, nz, angles, ns_extra, ds_ratio, seed):
    ns = max(1, nx + ns_extra)
    g = _geom(oracle, nx, ny, nz, angles, ns=ns, ds_ratio=ds_ratio)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nz, ny, nx))
    d = rng.standard_normal(g.data_shape)
    lhs = float(np.vdot(oracle.project(g, v), d))
    rhs = float(np.vdot(v, oracle.backproject(g, d)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(v) * np.linalg.norm(d))


@settings(**SETTINGS)
@given(n=st.integers(3, 10), nz=st.integers(1, 4), T=st.floats(0.02, 0.6), cfl=st.floats(0.05, 0.45),
       contrast=st.floats(0.0, 0.6), seed=st.integers(0, 2 ** 16))
def test_wave_transpose_dot_test_on_random_speeds(oracle, n, nz, T, cfl, contrast, seed):
    rng = np.random.default_rng(seed)
    shape = (nz, n, n + 1)
    c = 1.0 + contrast * rng.uniform(-1, 1, shape)
    g = oracle.Geometry(nx=n + 1, ny=n, nz=nz, dx=0.1, T=T, angles=np.zeros(1), cfl=cfl)
    h = rng.standard_normal(shape)
    q = rng.standard_normal(shape)
    lhs = float(np.vdot(oracle.wave(g, c, h), q))
    rhs = float(np.vdot(h, oracle.wave_T(g, c, q)))
    scale = np.linalg.norm(oracle.wave(g, c, h)) * np.linalg.norm(q) + abs(lhs)
    assert abs(lhs - rhs) <= 1e-11 * scale


@settings(**SETTINGS)
@given(ns=st.integers(1, 40), n_angles=st.integers(1, 5), seed=st.integers(0, 2 ** 16))
def test_ramp_symmetric_positive_definite_for_any_row_length(oracle, ns, n_angles, seed):
    g = _geom(oracle, ns, 3, 1, np.linspace(0, math.pi, n_angles, endpoint=False), ns=ns)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(g.data_shape)
    b = rng.standard_normal(g.data_shape)
    la, lb = oracle.ramp(g, a), oracle.ramp(g, b)
    assert abs(np.vdot(la, b) - np.vdot(a, lb)) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(b) * ns
    assert np.vdot(la, a) > 0.0


@settings(max_examples=6, deadline=None, derandomize=True)
@given(n=st.integers(4, 7), n_angles=st.integers(2, 5), lam=st.sampled_from([1e-3, 1e-1]),
       seed=st.integers(0, 2 ** 16))
def test_fb_with_positivity_stays_nonnegative_and_descends(oracle, n, n_angles, lam, seed):
    rng = np.random.default_rng(seed)
    shape = (2, n, n)
    c = 1.0 + 0.2 * rng.uniform(-1, 1, shape)
    g = oracle.Geometry(nx=n, ny=n, nz=2, dx=0.1, T=0.2, angles=np.linspace(0, math.pi, n_angles, endpoint=False))
    G = rng.standard_normal(g.data_shape)
    # s = 1/L with L from a long power iteration (L converges from below to the top eigenvalue)
    _, _, s_long = oracle.fb(g, c, G, lam, n_iter=0, n_power=400, flags=oracle.POSITIVITY | oracle.PRECOND)
    s = 0.99 * s_long
    h, obj, _ = oracle.fb(g, c, G, lam, step=s, n_iter=8, flags=oracle.POSITIVITY | oracle.PRECOND)
    assert np.all(h >= 0.0)
    assert np.all(np.diff(obj) <= 1e-12 * np.abs(obj[:-1]))

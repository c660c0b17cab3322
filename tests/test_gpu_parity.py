"""GPU parity: every operator of the HIP library against the FP64 oracle.

Inputs are seeded (synth), identical on both sides (FP32 cases feed the
oracle the FP32-rounded values).  Tolerances (relative L2):
  FP64: 1e-12 per operator, 1e-10 for reconstructions;
  FP32: 1e-5 for anything containing the wave solve, 2e-6 for X, X^T, Lambda,
        1e-4 for reconstructions after a fixed iteration count.
Grids are ragged on purpose (several 64-wide tiles plus a tail, odd ny, nz).
"""
import math

import numpy as np
import pytest

from conftest import rel_l2, rounded, to_dev, to_np
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
TOL_WAVE = {F32: 1e-5, F64: 1e-12}
TOL_X = {F32: 2e-6, F64: 1e-12}

SHAPES = [(23, 37, 70), (48, 48, 48), (9, 131, 67)]   # (nz, ny, nx)


def tol_xt(dtype, n_angles):
    """X^T sums n_angles terms per voxel (Sec. 3.1, X*).  In FP32 the rounding of a
    running sum of terms with random signs leaves a relative error of about
    u sqrt(n / 6) (u = 2^-24); the bound is 4 u sqrt(n), never below TOL_X and never
    above the 1e-5 required of the FP32 operators (reached at 1750 angles; measured
    5.9e-6 at 65535)."""
    if dtype == F64:
        return TOL_X[F64]
    return min(TOL_WAVE[F32], max(TOL_X[F32], 4 * 2.0 ** -24 * math.sqrt(n_angles)))


def make_case(shape, seed, n_angles=13, ns=None, ds_ratio=1.0, T=0.35, cfl=0.3):
    nz, ny, nx = shape
    dx = synth.grid_spacing(max(shape))
    rng = np.random.default_rng(seed)
    c = synth.sound_speed(shape, dx, rng, 3, 0.2, (0.8, 1.2))
    h = synth.gaussian_smooth(synth.balls(shape, dx, rng, 5), 1.0) + 0.1 * rng.standard_normal(shape)
    angles = np.sort(rng.uniform(0, math.pi, n_angles))
    angles[0] = 0.0
    if n_angles > 3:
        angles[1] = math.pi / 4
        angles[2] = math.pi / 2
    ns = ns or nx
    return dict(shape=shape, dx=dx, ds=ds_ratio * dx, ns=ns, T=T, cfl=cfl, c=c, h=h, angles=angles, rng=rng)


def oracle_geom(oracle, k, ndim=3):
    nz, ny, nx = k["shape"]
    return oracle.Geometry(nx=nx, ny=ny, nz=nz, dx=k["dx"], T=k["T"], angles=k["angles"], cfl=k["cfl"],
                           ns=k["ns"], ds=k["ds"], ndim=ndim)


def gpu_plan(k, dtype, naive=False, ndim=3, variant="pairs"):
    """variant: 'pairs' (two leapfrog steps per pass, forced), 'single' (one step per
    pass, forced), 'naive' (unblocked kernel)."""
    import paper_1901_06503_amd as ff
    if naive:
        variant = "naive"
    return ff.Plan(to_dev(k["c"], dtype), k["dx"], k["T"], k["angles"], ns=k["ns"], ds=k["ds"], cfl=k["cfl"],
                   ndim=ndim, naive_stencil=variant == "naive", two_step_stencil=variant == "pairs")

VARIANTS = ["pairs", "single", "naive"]


def _case_tag(shape, dtype, variant):
    print(f"[parity] shape={shape} dtype={dtype} variant={variant}", flush=True)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", SHAPES)
def test_plan_time_grid_matches_oracle(oracle, shape, dtype):
    k = make_case(shape, 1)
    with gpu_plan(k, dtype) as P:
        nt, dt, cmax = oracle.plan_info(oracle_geom(oracle, k), rounded(k["c"], dtype))
        assert P.nt == nt
        assert P.dt == dt
        assert P.cmax == cmax


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", SHAPES)
def test_wave_and_transpose(oracle, shape, dtype, variant):
    _case_tag(shape, dtype, variant)
    k = make_case(shape, 2)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    with gpu_plan(k, dtype, variant=variant) as P:
        p = to_np(P.wave(to_dev(h, dtype)))
        assert rel_l2(p, oracle.wave(g, c, h)) <= TOL_WAVE[dtype]
        q = to_np(P.wave_adjoint(to_dev(h, dtype)))
        assert rel_l2(q, oracle.wave_T(g, c, h)) <= TOL_WAVE[dtype]


# Grids where the two-step kernel splits z into several chunks of a length chosen
# from the resident work-group count, and picks its tile width per grid.  Expected
# launch shapes (tile width, height, planes per group) on 256 compute units:
# FP32 160^3 64 x 16, 16 chunks of 10 planes; FP32 224^3 128 x 16, 9 chunks of 25
# (last 24); FP64 192^3 64 x 16, 7 of 28 (last 24); FP32 96 x 250 x 250 (nz, ny, nx)
# 128 x 16 with ragged x and y tails (122 columns, 10 rows), 8 chunks of 12.
# 97 x 380 x 383: FP32 128 x 16 with 3 chunks of 33 (last 31) in one round, FP64
# 64 x 16 with 5 chunks of 20 (last 17, 720 groups: the chunk comes from the
# rounds x (planes + halo) estimate).  257 x 380 x 383 and x 382: FP32 128 x 16 with
# 7 chunks of 37 (last 35, 504 groups, two rounds).
# FP32 grids with even nx where the 128 x 16 tile is chosen run over pairs of
# x-adjacent points per lane (224^3, 96 x 250 x 250, 257 x 380 x 382), odd nx with
# one point per lane (97 and 257 x 380 x 383).
# Short solves (T = 0.04: n_t 8 to 22) keep the oracle quick.
MID_SIZES = [((160, 160, 160), F32, (64, 16, 10)), ((224, 224, 224), F32, (128, 16, 25)),
             ((192, 192, 192), F64, (64, 16, 28)), ((96, 250, 250), F32, (128, 16, 12)),
             ((97, 380, 383), F32, (128, 16, 33)), ((97, 380, 383), F64, (64, 16, 20)),
             ((257, 380, 383), F32, (128, 16, 37)), ((257, 380, 382), F32, (128, 16, 37))]


def _compute_units():
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("shape,dtype,launch", MID_SIZES,
                         ids=["f32-160", "f32-224", "f64-192", "f32-wide-ragged", "f32-odd-nx", "f64-rounds",
                              "f32-rounds", "f32-pairs-rounds"])
def test_wave_pairs_mid_size_chunking(oracle, shape, dtype, launch):
    _case_tag(shape, dtype, "pairs-auto")
    k = make_case(shape, 5, T=0.04)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    import paper_1901_06503_amd as ff
    with ff.Plan(to_dev(c, dtype), k["dx"], k["T"], k["angles"], cfl=k["cfl"], stencil_steps=2) as P:
        assert P.steps_per_pass == 2 and P.nt >= 5
        if _compute_units() == 256:
            assert P.stencil_shape == launch
        else:
            assert P.stencil_shape[0] in (64, 128)
        p = to_np(P.wave(to_dev(h, dtype)))
        assert rel_l2(p, oracle.wave(g, c, h)) <= TOL_WAVE[dtype]
        q = to_np(P.wave_adjoint(to_dev(h, dtype)))
        assert rel_l2(q, oracle.wave_T(g, c, h)) <= TOL_WAVE[dtype]


@pytest.mark.parametrize("nt", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("shape", [(40, 250, 250), (64, 130, 254)])
def test_pairs_of_points_every_step_count(oracle, shape, nt):
    """FP32 grids with even nx where the 128 x 16 tile is chosen run over pairs of
    x-adjacent points per lane: ragged x (125 and 127 pairs over 64-pair tiles) and y
    tails, several z-chunks, odd and even step counts."""
    _case_tag(shape, F32, f"pairs-of-points nt={nt}")
    k = make_case(shape, 17, n_angles=5)
    cmax = float(rounded(k["c"], F32).max())
    k["T"] = (nt - 0.5) * k["cfl"] * k["dx"] / cmax
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], F32), rounded(k["h"], F32)
    import paper_1901_06503_amd as ff
    with ff.Plan(to_dev(c, F32), k["dx"], k["T"], k["angles"], cfl=k["cfl"], stencil_steps=2) as P:
        assert P.nt == nt and P.steps_per_pass == 2
        if _compute_units() == 256:
            assert P.stencil_shape == (128, 16, 8)
        assert rel_l2(to_np(P.wave(to_dev(h, F32))), oracle.wave(g, c, h)) <= TOL_WAVE[F32]
        assert rel_l2(to_np(P.wave_adjoint(to_dev(h, F32))), oracle.wave_T(g, c, h)) <= TOL_WAVE[F32]


def test_pairs_of_points_with_buffers_at_odd_float_offsets(oracle):
    """The pairs-of-points form moves 8 bytes per lane; caller buffers that start at
    an odd float (contiguous views one float into an allocation) take the one-point
    form.  Forward with n_t = 5 reads the input as p(k-1) in its first pair and writes
    the output in its last; the adjoint writes its output in the last single step.
    The one-point form's launches give the same bits as the pairs form's."""
    shape = (40, 250, 250)
    _case_tag(shape, F32, "pairs-of-points odd offsets")
    k = make_case(shape, 19, n_angles=5)
    cmax = float(rounded(k["c"], F32).max())
    k["T"] = 4.5 * k["cfl"] * k["dx"] / cmax
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], F32), rounded(k["h"], F32)
    n = h.size
    import paper_1901_06503_amd as ff
    with ff.Plan(to_dev(c, F32), k["dx"], k["T"], k["angles"], cfl=k["cfl"], stencil_steps=2) as P:
        assert P.nt == 5 and P.steps_per_pass == 2
        hin = torch.zeros(n + 1, dtype=F32, device="cuda")[1:].view(shape)
        hin.copy_(to_dev(h, F32))
        out = torch.zeros(n + 1, dtype=F32, device="cuda")[1:].view(shape)
        assert hin.data_ptr() % 8 == 4 and out.data_ptr() % 8 == 4
        P.wave(hin, out=out)
        assert rel_l2(to_np(out), oracle.wave(g, c, h)) <= TOL_WAVE[F32]
        # aligned buffers: every pair launch takes the pairs form.  Both forms add each
        # point's neighbours in the same order, so the results are equal bit for bit.
        assert torch.equal(P.wave(to_dev(h, F32)), out)
        P.wave_adjoint(hin, out=out)
        assert rel_l2(to_np(out), oracle.wave_T(g, c, h)) <= TOL_WAVE[F32]
        assert torch.equal(P.wave_adjoint(to_dev(h, F32)), out)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_stencil_shape_of_one_step_and_naive_plans(dtype):
    """ffpat_plan_stencil_shape for the other two stencil kernels: the one-step
    kernel's 64 x 8 tile with one plane per work-group on a 48^3 grid (about 2048
    groups would need fewer), and zeros for the unblocked kernel."""
    k = make_case((48, 48, 48), 6)
    with gpu_plan(k, dtype, variant="single") as P:
        assert P.steps_per_pass == 1 and P.stencil_shape == (64, 8, 1)
    with gpu_plan(k, dtype, variant="naive") as P:
        assert P.stencil_shape == (0, 0, 0)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ds_ratio,ns_extra", [(1.0, 0), (0.83, 7), (1.3, -5)])
def test_project_backproject(oracle, shape, dtype, ds_ratio, ns_extra):
    nz, ny, nx = shape
    k = make_case(shape, 3, n_angles=17, ns=nx + ns_extra, ds_ratio=ds_ratio)
    g = oracle_geom(oracle, k)
    v = rounded(k["h"], dtype)
    d = rounded(k["rng"].standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype) as P:
        gp = to_np(P.project(to_dev(v, dtype)))
        assert rel_l2(gp, oracle.project(g, v)) <= TOL_X[dtype]
        bp = to_np(P.backproject(to_dev(d, dtype)))
        assert rel_l2(bp, oracle.backproject(g, d)) <= tol_xt(dtype, len(k["angles"]))


LDS_LAYOUTS = {
    # (nz, ny, nx), ns, angles
    "wide": ((5, 40, 300), 301, np.linspace(0.0, math.pi, 9, endpoint=False) + 0.05),
    "rows_only": ((6, 30, 50), 50, np.concatenate([np.linspace(0.0, 0.7, 6), np.linspace(2.45, 3.1, 5)])),
    "cols_only": ((6, 30, 50), 50, np.linspace(0.9, 2.2, 11)),
    "many_angles": ((7, 33, 35), 35, np.linspace(0.0, math.pi, 100, endpoint=False)),
    # the largest detector rows and angle count the boundary accepts: 8192 bins on 4
    # planes (FP32: the staged backprojector holds one angle's rows per chunk; FP64:
    # the L2 kernel), on 8 planes (FP32 8-plane projector, L2 backprojector), and
    # 65535 angles
    "widest_detector_4": ((4, 9, 11), 8192, np.linspace(0.0, math.pi, 5, endpoint=False) + 0.1),
    "widest_detector_8": ((8, 9, 11), 8192, np.linspace(0.0, math.pi, 5, endpoint=False) + 0.1),
    "most_angles": ((4, 9, 11), 11, np.linspace(0.0, math.pi, 65535, endpoint=False)),
}


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("layout", sorted(LDS_LAYOUTS))
def test_project_backproject_work_decompositions(oracle, dtype, layout):
    """X and X^T where the staged kernels split the work unevenly: more than 256
    bins (two bin blocks, lines longer than one LDS chunk), angle sets of one
    orientation only, more than 32 angles per orientation, plane counts that
    are not multiples of 4."""
    shape, ns, angles = LDS_LAYOUTS[layout]
    k = make_case(shape, 31, n_angles=len(angles), ns=ns)
    k["angles"] = np.asarray(angles, dtype=np.float64)
    g = oracle_geom(oracle, k)
    v = rounded(k["h"], dtype)
    d = rounded(k["rng"].standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype) as P:
        gp = to_np(P.project(to_dev(v, dtype)))
        assert rel_l2(gp, oracle.project(g, v)) <= TOL_X[dtype]
        bp = to_np(P.backproject(to_dev(d, dtype)))
        assert rel_l2(bp, oracle.backproject(g, d)) <= tol_xt(dtype, len(angles))


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("ns,ds_ratio", [(1, 1.0), (2, 1.0), (9, 1.0), (16, 1.0), (48, 1.0), (257, 1.0), (700, 1.0),
                                         (2047, 1.0), (2048, 1.0), (2049, 1.0), (8192, 1.0), (48, 0.83), (257, 1.3)])
def test_ramp(oracle, dtype, ns, ds_ratio):
    """Rows of up to 2048 bins take the register-window kernel (several rows per
    work-group below 129 bins; one row of 256 threads at 2041..2048), longer rows
    the one-row fallback, up to the largest accepted row (8192 bins).  Detector
    spacings off the grid spacing check the filter's scale, pi / (N_angles dx^2)
    for any ds."""
    k = make_case((5, 8, 8), 4, n_angles=7, ns=ns, ds_ratio=ds_ratio)
    g = oracle_geom(oracle, k)
    r = rounded(k["rng"].standard_normal(g.data_shape), dtype)
    ref = oracle.ramp(g, r)
    with gpu_plan(k, dtype) as P:
        y = to_np(P.ramp(to_dev(r, dtype)))
        assert rel_l2(y, ref) <= TOL_X[dtype]
        # in place
        t = to_dev(r, dtype)
        P.ramp(t, out=t)
        assert rel_l2(to_np(t), ref) <= TOL_X[dtype]


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", SHAPES[:2])
def test_forward_adjoint(oracle, shape, dtype):
    k = make_case(shape, 5, n_angles=19)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    d = rounded(k["rng"].standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype) as P:
        A = to_np(P.forward(to_dev(h, dtype)))
        assert rel_l2(A, oracle.forward(g, c, h)) <= TOL_WAVE[dtype]
        AT = to_np(P.adjoint(to_dev(d, dtype)))
        assert rel_l2(AT, oracle.adjoint(g, c, d)) <= TOL_WAVE[dtype]


def test_gpu_dot_test_fp64():
    k = make_case((31, 40, 66), 6, n_angles=23)
    h = k["h"]
    d = k["rng"].standard_normal((23, 31, 66))
    with gpu_plan(k, F64) as P:
        lhs = float(torch.sum(P.forward(to_dev(h, F64)) * to_dev(d, F64)))
        rhs = float(torch.sum(to_dev(h, F64) * P.adjoint(to_dev(d, F64))))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("dtype", [F64, F32])
def test_edge_single_step_single_angle_single_plane(oracle, dtype):
    # n_t = 1 (tiny T), one angle, one z plane, ns = 1
    k = make_case((1, 12, 10), 7, n_angles=1, ns=1, T=0.005)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    d = rounded(k["rng"].standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype) as P:
        assert P.nt == 1
        assert rel_l2(to_np(P.forward(to_dev(h, dtype))), oracle.forward(g, c, h)) <= TOL_WAVE[dtype]
        assert rel_l2(to_np(P.adjoint(to_dev(d, dtype))), oracle.adjoint(g, c, d)) <= TOL_WAVE[dtype]


@pytest.mark.parametrize("dtype", [F64, F32])
def test_edge_two_steps_and_tiny_grid(oracle, dtype):
    k = make_case((3, 2, 5), 8, n_angles=4)
    k["T"] = 1.5 * k["cfl"] * k["dx"] / float(rounded(k["c"], dtype).max())   # between one and two steps
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    with gpu_plan(k, dtype) as P:
        assert P.nt == 2
        assert rel_l2(to_np(P.wave(to_dev(h, dtype))), oracle.wave(g, c, h)) <= TOL_WAVE[dtype]
        assert rel_l2(to_np(P.wave_adjoint(to_dev(h, dtype))), oracle.wave_T(g, c, h)) <= TOL_WAVE[dtype]


THIN = [(6, 7, 1), (6, 1, 9), (1, 1, 1), (5, 1, 1), (1, 1, 8)]   # (nz, ny, nx)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("shape", THIN)
def test_edge_grids_one_voxel_wide(oracle, shape, dtype, variant):
    """Grids one voxel wide in x and/or y (and a single voxel): every stencil
    neighbour but the centre lies outside, where the field is zero; n_t = 5 (first
    step, pairs, a single-step tail); one detector bin per row when nx = 1."""
    _case_tag(shape, dtype, variant)
    dx = synth.grid_spacing(12)
    rng = np.random.default_rng(71)
    k = dict(shape=shape, dx=dx, ds=dx, ns=shape[2], T=0.35, cfl=0.3, c=1.0 + 0.1 * rng.standard_normal(shape),
             h=rng.standard_normal(shape), angles=np.array([0.0, 0.7, math.pi / 2, 2.4]), rng=rng)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    d = rounded(rng.standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype, variant=variant) as P:
        assert P.nt == 5
        assert rel_l2(to_np(P.forward(to_dev(h, dtype))), oracle.forward(g, c, h)) <= TOL_WAVE[dtype]
        assert rel_l2(to_np(P.adjoint(to_dev(d, dtype))), oracle.adjoint(g, c, d)) <= TOL_WAVE[dtype]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", [F64, F32])
def test_edge_most_planes(oracle, dtype, variant):
    """nz = 65535, the most planes the boundary accepts (the unblocked stencil and the
    projector's plane copies launch one grid layer per plane)."""
    shape = (65535, 2, 3)
    _case_tag(shape, dtype, variant)
    dx = synth.grid_spacing(12)
    rng = np.random.default_rng(73)
    k = dict(shape=shape, dx=dx, ds=dx, ns=3, T=0.35, cfl=0.3, c=1.0 + 0.1 * rng.standard_normal(shape),
             h=rng.standard_normal(shape), angles=np.array([0.0, 0.7, math.pi / 2, 2.4]), rng=rng)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    d = rounded(rng.standard_normal(g.data_shape), dtype)
    with gpu_plan(k, dtype, variant=variant) as P:
        assert P.nt == 7
        assert rel_l2(to_np(P.forward(to_dev(h, dtype))), oracle.forward(g, c, h)) <= TOL_WAVE[dtype]
        assert rel_l2(to_np(P.adjoint(to_dev(d, dtype))), oracle.adjoint(g, c, d)) <= TOL_WAVE[dtype]


@pytest.mark.parametrize("variant", ["pairs", "single"])
@pytest.mark.parametrize("nt", [1, 2, 3, 4, 5, 6, 7])
def test_every_step_count(oracle, nt, variant):
    """n_t = 1..7 covers first step only, pairs, odd leftovers and the dividing last step."""
    k = make_case((13, 19, 70), 13, n_angles=5)
    cmax = float(rounded(k["c"], F64).max())
    k["T"] = (nt - 0.5) * k["cfl"] * k["dx"] / cmax
    g = oracle_geom(oracle, k)
    c, h = k["c"], k["h"]
    d = k["rng"].standard_normal(g.data_shape)
    with gpu_plan(k, F64, variant=variant) as P:
        assert P.nt == nt
        assert rel_l2(to_np(P.wave(to_dev(h, F64))), oracle.wave(g, c, h)) <= 1e-12
        assert rel_l2(to_np(P.wave_adjoint(to_dev(h, F64))), oracle.wave_T(g, c, h)) <= 1e-12
        assert rel_l2(to_np(P.forward(to_dev(h, F64))), oracle.forward(g, c, h)) <= 1e-12
        assert rel_l2(to_np(P.adjoint(to_dev(d, F64))), oracle.adjoint(g, c, d)) <= 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", [F64, F32])
def test_two_dimensional_mode(oracle, dtype, variant):
    k = make_case((11, 50, 66), 9, n_angles=11)
    g = oracle_geom(oracle, k, ndim=2)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    with gpu_plan(k, dtype, ndim=2, variant=variant) as P:
        assert rel_l2(to_np(P.wave(to_dev(h, dtype))), oracle.wave(g, c, h)) <= TOL_WAVE[dtype]
        assert rel_l2(to_np(P.forward(to_dev(h, dtype))), oracle.forward(g, c, h)) <= TOL_WAVE[dtype]


# ---------------------------------------------------------------- Algorithm 8
def _fb_case(oracle, shape, n_angles, seed, dtype, eta=0.01, ds_ratio=1.0, ns_extra=0):
    k = make_case(shape, seed, n_angles=n_angles, T=0.5, ds_ratio=ds_ratio, ns=shape[2] + ns_extra)
    k["h"] = np.abs(k["h"])
    g = oracle_geom(oracle, k)
    c = rounded(k["c"], dtype)
    clean = oracle.forward(g, c, rounded(k["h"], dtype))
    G = clean + eta * np.mean(clean) * k["rng"].standard_normal(clean.shape)
    return k, g, c, rounded(G, dtype)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("ds_ratio,ns_extra", [(1.0, 0), (0.83, 7), (1.3, -5)])
def test_reconstruct_matches_oracle(oracle, dtype, ds_ratio, ns_extra):
    """Algorithm 8 with the ramp preconditioner; detector spacings 0.83 dx (footprints
    over several bins) and 1.3 dx put the filter's scale and the multi-bin
    backprojection inside the iteration and the power-iteration step."""
    k, g, c, G = _fb_case(oracle, (20, 26, 30), 16, 10, dtype, ds_ratio=ds_ratio, ns_extra=ns_extra)
    lam, K = 1e-3, 5
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, step=0.0, n_iter=K, n_power=20,
                                      flags=oracle.POSITIVITY | oracle.PRECOND)
    with gpu_plan(k, dtype) as P:
        res = P.reconstruct(to_dev(G, dtype), lam, K, step=0.0, n_power=20)
    tol = 1e-10 if dtype == F64 else 1e-4
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


def test_pairs_of_points_reconstruction_in_graphs(oracle):
    """Algorithm 8 in FP32 on a grid where the plan takes the pairs-of-points form,
    its power iteration and FB iterations replayed from captured graphs."""
    shape = (40, 250, 250)
    _case_tag(shape, F32, "pairs-of-points reconstruct")
    k = make_case(shape, 23, n_angles=6)
    cmax = float(rounded(k["c"], F32).max())
    k["T"] = 6.5 * k["cfl"] * k["dx"] / cmax
    k["h"] = np.abs(k["h"])
    g = oracle_geom(oracle, k)
    c = rounded(k["c"], F32)
    clean = oracle.forward(g, c, rounded(k["h"], F32))
    G = rounded(clean + 0.01 * np.mean(clean) * k["rng"].standard_normal(clean.shape), F32)
    lam, K = 1e-3, 4
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, step=0.0, n_iter=K, n_power=6,
                                      flags=oracle.POSITIVITY | oracle.PRECOND)
    import paper_1901_06503_amd as ff
    with ff.Plan(to_dev(c, F32), k["dx"], k["T"], k["angles"], cfl=k["cfl"], stencil_steps=2) as P:
        assert P.nt == 7 and P.steps_per_pass == 2
        if _compute_units() == 256:
            assert P.stencil_shape == (128, 16, 8)
        res = P.reconstruct(to_dev(G, F32), lam, K, step=0.0, n_power=6)
    assert res.step == pytest.approx(s_ref, rel=1e-4)
    assert rel_l2(to_np(res.h), h_ref) <= 1e-4
    assert np.allclose(res.objective, obj_ref, rtol=1e-4, atol=0)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_reconstruct_masks_and_fixed_step(oracle, dtype):
    k, g, c, G = _fb_case(oracle, (12, 21, 34), 9, 11, dtype)
    sup = np.zeros(g.vol_shape, dtype=np.uint8)
    sup[2:-2, 3:-3, 4:-4] = 1
    det = np.ones(g.data_shape, dtype=np.uint8)
    det[:, :, 14:20] = 0
    h_ref, obj_ref, _ = oracle.fb(g, c, G, 0.05, step=0.02, n_iter=4, flags=oracle.PRECOND,
                                  support=sup, det_mask=det)
    with gpu_plan(k, dtype) as P:
        res = P.reconstruct(to_dev(G, dtype), 0.05, 4, step=0.02, positivity=False,
                            support=torch.from_numpy(sup).cuda(), det_mask=torch.from_numpy(det).cuda())
    tol = 1e-10 if dtype == F64 else 1e-4
    assert res.step == 0.02
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_reconstruct_resume_is_bitwise_continuous(dtype):
    # (h, k, s) is the whole state: 2 + 3 iterations from the stored step == 5 iterations
    k = make_case((10, 16, 20), 12, n_angles=8)
    G = to_dev(np.abs(k["rng"].standard_normal((8, 10, 20))), dtype)
    with gpu_plan(k, dtype) as P:
        full = P.reconstruct(G, 1e-3, 5)
        part = P.reconstruct(G, 1e-3, 2)
        part2 = P.reconstruct(G, 1e-3, 3, h0=part.h, use_plan_step=True)
    assert part2.step == full.step
    assert torch.equal(part2.h, full.h)
    assert np.array_equal(np.concatenate([part.objective, part2.objective]), full.objective)

"""Three leapfrog steps per stencil pass (eq. wave1): wave_step3_wide for FP32 (pairs
of x-adjacent points, 1024 threads, one interior point and one ring point per
thread), wave_step3_split for FP64.

A kernel computes p(k+1), p(k+2), p(k+3) from p(k-1), p(k) and k' in one pass and
adds each point's neighbours in the same order as the one- and two-step kernels, so
a solve with three steps per pass must equal the same solve with two steps per
pass bit for bit, and the oracle within the operator tolerances.  Cases: every chain
length from 1 to 11 leapfrog levels (triples plus a pair or a single pass, the
adjoint's dividing last step alone), FP32 over pairs of x-adjacent points on ragged
grids (even nx, 128 x 16 tiles) and FP64 on ragged and degenerate grids (one voxel
wide in x, y or z), several z-chunks and rounds of work-groups, caller buffers off
8-byte alignment (the three-step kernel is then not taken), Algorithm 8 with
captured graphs, the 256^3 workload, the serving loop, and the default plans of the
96^3..160^3 grids that take three steps per pass with 3- to 14-plane chunks.
"""
import numpy as np
import pytest

from conftest import rel_l2, rounded, to_dev, to_np
from test_gpu_parity import TOL_WAVE, make_case, oracle_geom

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


def _tag(shape, dtype, what):
    print(f"[triple] shape={shape} dtype={dtype} {what}", flush=True)


def _plan(k, dtype, steps):
    import paper_1901_06503_amd as ff
    return ff.Plan(to_dev(rounded(k["c"], dtype), dtype), k["dx"], k["T"], k["angles"], ns=k["ns"], ds=k["ds"],
                   cfl=k["cfl"], stencil_steps=steps)


def _with_nt(k, dtype, nt):
    cmax = float(rounded(k["c"], dtype).max())
    k["T"] = (nt - 0.5) * k["cfl"] * k["dx"] / cmax
    return k


def _check(oracle, k, dtype, nt=None):
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], dtype), rounded(k["h"], dtype)
    with _plan(k, dtype, 3) as P3, _plan(k, dtype, 2) as P2:
        assert P3.steps_per_pass == 3 and P2.steps_per_pass == 2
        if nt is not None:
            assert P3.nt == nt
        hd = to_dev(h, dtype)
        f3, f2 = P3.wave(hd), P2.wave(hd)
        a3, a2 = P3.wave_adjoint(hd), P2.wave_adjoint(hd)
    assert torch.equal(f3, f2), "three steps per pass differ from two"
    assert torch.equal(a3, a2), "three steps per pass differ from two (adjoint)"
    assert rel_l2(to_np(f3), oracle.wave(g, c, h)) <= TOL_WAVE[dtype]
    assert rel_l2(to_np(a3), oracle.wave_T(g, c, h)) <= TOL_WAVE[dtype]


@pytest.mark.parametrize("nt", [1, 2, 3, 4, 5, 6, 7, 8, 10, 11])
@pytest.mark.parametrize("shape", [(40, 250, 250), (64, 130, 254)])
def test_f32_pairs_every_chain_length(oracle, shape, nt):
    """FP32, even nx, the 128 x 16 tile: ragged x (125 and 127 pairs over 64-pair
    tiles) and y tails, several z-chunks."""
    _tag(shape, F32, f"nt={nt}")
    k = _with_nt(make_case(shape, 31, n_angles=5), F32, nt)
    _check(oracle, k, F32, nt)


@pytest.mark.parametrize("nt", [3, 4, 5, 7, 10])
@pytest.mark.parametrize("shape", [(23, 37, 70), (48, 48, 48), (9, 131, 67)])
def test_f64_every_chain_length(oracle, shape, nt):
    _tag(shape, F64, f"nt={nt}")
    k = _with_nt(make_case(shape, 32, n_angles=5), F64, nt)
    _check(oracle, k, F64, nt)


@pytest.mark.parametrize("shape", [(6, 5, 1), (7, 1, 9), (1, 8, 11), (1, 1, 1), (3, 2, 5), (70, 17, 3),
                                   (65535, 2, 3)])
def test_f64_degenerate_grids(oracle, shape):
    """Grids one voxel wide in x, y or z (every neighbour beyond the grid is zero), a
    single voxel, a tall thin grid with several z-chunks, and the most planes the
    boundary accepts."""
    import synth
    _tag(shape, F64, "degenerate")
    dx = synth.grid_spacing(12)
    rng = np.random.default_rng(75)
    k = dict(shape=shape, dx=dx, ds=dx, ns=shape[2], T=0.35, cfl=0.3, c=1.0 + 0.1 * rng.standard_normal(shape),
             h=rng.standard_normal(shape), angles=np.array([0.0, 0.7, 2.4]), rng=rng)
    k = _with_nt(k, F64, 7)
    _check(oracle, k, F64, 7)


# Grids with several z-chunks (and, for the last two, more than one round of
# work-groups on 256 compute units); short solves (T = 0.04) keep the oracle quick.
MID = [((224, 224, 224), F32), ((96, 250, 250), F32), ((257, 380, 382), F32), ((192, 192, 192), F64),
       ((97, 380, 383), F64)]


@pytest.mark.parametrize("shape,dtype", MID, ids=["f32-224", "f32-ragged", "f32-rounds", "f64-192", "f64-rounds"])
def test_mid_size_chunking(oracle, shape, dtype):
    _tag(shape, dtype, "mid-size")
    k = make_case(shape, 34, n_angles=5, T=0.04)
    _check(oracle, k, dtype)


def test_buffers_off_alignment_take_smaller_passes(oracle):
    """The three-step kernel moves 8-byte elements; caller buffers one float off
    8-byte alignment make its chain take the two-step kernel's one-point form for
    the launches that touch them: the same bits as aligned buffers."""
    shape = (40, 250, 250)
    _tag(shape, F32, "odd offsets")
    k = _with_nt(make_case(shape, 35, n_angles=5), F32, 8)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], F32), rounded(k["h"], F32)
    n = h.size
    with _plan(k, F32, 3) as P:
        assert P.nt == 8 and P.steps_per_pass == 3
        hin = torch.zeros(n + 1, dtype=F32, device="cuda")[1:].view(shape)
        hin.copy_(to_dev(h, F32))
        out = torch.zeros(n + 1, dtype=F32, device="cuda")[1:].view(shape)
        assert hin.data_ptr() % 8 == 4 and out.data_ptr() % 8 == 4
        P.wave(hin, out=out)
        assert torch.equal(P.wave(to_dev(h, F32)), out)
        assert rel_l2(to_np(out), oracle.wave(g, c, h)) <= TOL_WAVE[F32]
        P.wave_adjoint(hin, out=out)
        assert torch.equal(P.wave_adjoint(to_dev(h, F32)), out)
        assert rel_l2(to_np(out), oracle.wave_T(g, c, h)) <= TOL_WAVE[F32]


@pytest.mark.parametrize("dtype", [F32, F64])
def test_reconstruction_in_graphs(oracle, dtype):
    """Algorithm 8 (Sec. 3.2) with three steps per pass, power iteration and FB
    iterations replayed from captured graphs: the oracle's step, iterate and
    objective history, and the bits of the two-step plan."""
    shape = (40, 250, 250) if dtype == F32 else (20, 70, 90)
    _tag(shape, dtype, "reconstruct")
    k = _with_nt(make_case(shape, 36, n_angles=6), dtype, 10)
    k["h"] = np.abs(k["h"])
    g = oracle_geom(oracle, k)
    c = rounded(k["c"], dtype)
    clean = oracle.forward(g, c, rounded(k["h"], dtype))
    G = rounded(clean + 0.01 * np.mean(clean) * k["rng"].standard_normal(clean.shape), dtype)
    lam, K = 1e-3, 4
    h_ref, obj_ref, s_ref = oracle.fb(g, c, G, lam, step=0.0, n_iter=K, n_power=6,
                                      flags=oracle.POSITIVITY | oracle.PRECOND)
    res = {}
    for steps in (3, 2):
        with _plan(k, dtype, steps) as P:
            assert P.nt == 10 and P.steps_per_pass == steps
            res[steps] = P.reconstruct(to_dev(G, dtype), lam, K, step=0.0, n_power=6)
    tol = 1e-4 if dtype == F32 else 1e-10
    r = res[3]
    assert r.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(r.h), h_ref) <= tol
    assert np.allclose(r.objective, obj_ref, rtol=tol, atol=0)
    assert torch.equal(r.h, res[2].h) and r.step == res[2].step
    assert np.array_equal(r.objective, res[2].objective)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_256cubed_workload_equals_two_steps(dtype):
    """The benchmark's wave solves (256^3, T = 0.5, n_t 171 / 170): three steps per
    pass give the bits of two steps per pass, whose parity with the oracle the
    full-size tests establish."""
    import paper_1901_06503_amd as ff
    import synth
    case = synth.make_case("c256", 3001)
    _tag((256, 256, 256), dtype, "256^3")
    c = to_dev(rounded(case.c, dtype), dtype)
    h = to_dev(rounded(case.h_true, dtype), dtype)
    with ff.Plan(c, case.dx, case.T, case.angles, stencil_steps=3) as P3, \
            ff.Plan(c, case.dx, case.T, case.angles, stencil_steps=2) as P2:
        assert P3.steps_per_pass == 3 and P3.nt == P2.nt
        assert torch.equal(P3.wave(h), P2.wave(h))
        assert torch.equal(P3.wave_adjoint(h), P2.wave_adjoint(h))


def test_serving_mix_with_three_step_plans():
    """The serving loop on jobs whose plans run three steps per pass (FP32, 40 x 250 x
    250, plans reused across jobs, captured graphs replayed on the jobs' streams): every
    job's result in the mix equals its result alone, bit for bit.  All four arrive at
    once and two are admitted at a time, so two run together whatever the jobs' speed
    (each takes a few ms) and the last two take over the first two's plans."""
    import paper_1901_06503_amd as ff
    from paper_1901_06503_amd.serving import Job, Scheduler, run_serial
    shape = (40, 250, 250)
    _tag(shape, F32, "serving")
    jobs = []
    angles = None
    for i in range(4):
        k = make_case(shape, 40 + i, n_angles=6, T=0.1)
        angles = k["angles"] if angles is None else angles     # one geometry: plans are reused
        c = to_dev(rounded(k["c"], F32), F32)
        with ff.Plan(c, k["dx"], k["T"], angles) as P:
            assert P.steps_per_pass == 3
            G = P.forward(to_dev(rounded(np.abs(k["h"]), F32), F32))
        torch.cuda.synchronize()
        jobs.append(Job(job_id=i, arrival=0.0, c=c.cpu().pin_memory(), G=G.cpu().pin_memory(), dx=k["dx"],
                        T=k["T"], angles=angles, lam=1e-3, n_iter=4, n_power=3))

    def clone():
        return [Job(job_id=j.job_id, arrival=j.arrival, c=j.c, G=j.G, dx=j.dx, T=j.T, angles=j.angles, lam=j.lam,
                    n_iter=j.n_iter, n_power=j.n_power) for j in jobs]

    alone = sorted(run_serial(clone()), key=lambda j: j.job_id)
    with Scheduler(hbm_budget=8 << 30, max_active=2, iters_per_turn=2, low_concurrency=2) as sched:
        mixed = sorted(sched.run(clone()), key=lambda j: j.job_id)
    assert sched.peak_running > 1 and sched.plans_reused > 0
    for a, b in zip(alone, mixed):
        assert a.status == b.status == "done"
        assert a.step == b.step
        assert torch.equal(a.h, b.h)
        assert np.array_equal(np.array(a.objective), np.array(b.objective))


# FP32 grids that take three steps per pass by default where the two-step rule keeps
# the 64-point tile or one step per pass, with the z-chunk the plan picks on 256
# compute units (one round of groups: 3 or 4 planes up to 128^3)
DEFAULT_MID = [((96, 96, 96), 3), ((112, 112, 112), 4), ((128, 128, 128), 4), ((160, 160, 160), 14)]


@pytest.mark.parametrize("shape,zchunk", DEFAULT_MID, ids=["96", "112", "128", "160"])
def test_default_plan_takes_three_steps_on_mid_grids(oracle, shape, zchunk):
    """Default FP32 plans on these grids run wave_step3_wide with short z-chunks; their
    solves equal those of a plan forced to two steps per pass bit for bit and the
    oracle within the FP32 operator tolerance (n_t = 11: three passes of three steps,
    then a pass of two; the adjoint ends with its dividing step alone)."""
    import paper_1901_06503_amd as ff
    _tag(shape, F32, "default three-step plan")
    k = _with_nt(make_case(shape, 37, n_angles=3), F32, 11)
    g = oracle_geom(oracle, k)
    c, h = rounded(k["c"], F32), rounded(k["h"], F32)
    with ff.Plan(to_dev(c, F32), k["dx"], k["T"], k["angles"], cfl=k["cfl"]) as P, _plan(k, F32, 2) as P2:
        assert P.nt == 11 and P.steps_per_pass == 3 and P2.steps_per_pass == 2
        if torch.cuda.get_device_properties(0).multi_processor_count == 256:
            assert P.stencil_shape == (128, 16, zchunk)
        hd = to_dev(h, F32)
        f3, f2 = P.wave(hd), P2.wave(hd)
        a3, a2 = P.wave_adjoint(hd), P2.wave_adjoint(hd)
    assert torch.equal(f3, f2) and torch.equal(a3, a2)
    assert rel_l2(to_np(f3), oracle.wave(g, c, h)) <= TOL_WAVE[F32]
    assert rel_l2(to_np(a3), oracle.wave_T(g, c, h)) <= TOL_WAVE[F32]

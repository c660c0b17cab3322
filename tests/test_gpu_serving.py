"""Serving loop and captured graphs.

* Graph replays equal eager launches bitwise (deterministic kernels, no
  atomics), across several replays with other eager work in between.
* The asynchronous enqueue/report pair equals ffpat_reconstruct.
* Continuous batching: every job's result in the mix equals its result alone
  (bitwise), admission never exceeds the HBM budget, a failing job does not
  disturb the others.
"""
import math

import numpy as np
import pytest

from conftest import to_dev
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(n, n_angles, seed, dtype=torch.float32):
    dx = synth.grid_spacing(n)
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    c = synth.sound_speed(shape, dx, rng, 2, 0.2, (0.8, 1.2))
    h = synth.gaussian_smooth(synth.balls(shape, dx, rng, 4), 1.0)
    angles = synth.uniform_angles(n_angles)
    return dx, angles, to_dev(c, dtype), to_dev(h, dtype), rng


def _data(plan, h, rng):
    g = plan.forward(h)
    noise = torch.from_numpy(rng.standard_normal(plan.data_shape)).to(g.device, g.dtype)
    return g + 0.02 * float(g.double().mean()) * noise


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_graph_replay_equals_eager(dtype):
    import paper_1901_06503_amd as ff
    dx, angles, c, h, rng = _inputs(40, 24, 61, dtype)
    with ff.Plan(c, dx, 0.5, angles, use_graphs=True) as Pg, ff.Plan(c, dx, 0.5, angles, use_graphs=False) as Pe:
        G = _data(Pe, h, rng)
        for n_iter in (3, 1, 4):
            rg = Pg.reconstruct(G, 1e-3, n_iter)
            _ = Pe.forward(h)                                  # eager work between replays
            torch.cuda.synchronize()
            re = Pe.reconstruct(G, 1e-3, n_iter)
            assert rg.step == re.step
            assert torch.equal(rg.h, re.h)
            assert np.array_equal(rg.objective, re.objective)
        # a new iterate buffer forces a re-capture; results still match
        h0 = torch.zeros_like(h)
        rg = Pg.reconstruct(G, 1e-3, 2, h0=h0)
        re = Pe.reconstruct(G, 1e-3, 2)
        assert torch.equal(rg.h, re.h)


def test_longer_run_after_a_captured_one_records_its_objective():
    # 3 iterations capture the iteration graph with the plan's first objective buffer
    # (1024 values); 1100 iterations with the same G and iterate buffer move it.  The
    # graph must be captured again: results, history and step equal eager launches.
    import paper_1901_06503_amd as ff
    dx, angles, c, h, rng = _inputs(24, 12, 67)
    with ff.Plan(c, dx, 0.5, angles, use_graphs=True) as Pg, ff.Plan(c, dx, 0.5, angles, use_graphs=False) as Pe:
        G = _data(Pe, h, rng)
        hg, he = torch.zeros_like(h), torch.zeros_like(h)
        for n_iter, plan_step in ((3, False), (1100, True)):
            rg = Pg.reconstruct(G, 1e-3, n_iter, h0=hg, use_plan_step=plan_step)
            re = Pe.reconstruct(G, 1e-3, n_iter, h0=he, use_plan_step=plan_step)
            assert rg.step == re.step
            assert torch.equal(rg.h, re.h)
            assert np.array_equal(rg.objective, re.objective)
            assert np.all(np.isfinite(rg.objective)) and rg.objective[-1] <= rg.objective[0]


def test_enqueue_report_equals_reconstruct():
    import paper_1901_06503_amd as ff
    dx, angles, c, h, rng = _inputs(32, 16, 62)
    with ff.Plan(c, dx, 0.5, angles) as P:
        G = _data(P, h, rng)
        ref = P.reconstruct(G, 1e-3, 6)
        x = torch.zeros_like(h)
        P.fb_enqueue(G, 1e-3, 0, x)
        P.fb_enqueue(G, 1e-3, 4, x, use_plan_step=True)
        s1, o1 = P.fb_report(4)
        P.fb_enqueue(G, 1e-3, 2, x, use_plan_step=True)
        s2, o2 = P.fb_report(2)
    assert s1 == s2 == ref.step
    assert torch.equal(x, ref.h)
    assert np.array_equal(np.concatenate([o1, o2]), ref.objective)


def test_set_speed_equals_a_new_plan():
    """ffpat_plan_set_speed: a plan given a new sound speed reconstructs bit for bit as a
    plan created with it, with the captured graphs kept (same n_t) or re-captured (a
    faster medium takes more steps); an invalid speed is rejected and leaves the plan's
    time grid as it was."""
    import paper_1901_06503_amd as ff
    dx, angles, c1, h, rng = _inputs(36, 20, 63)
    c2 = c1.flip(0).contiguous()                          # same range, same n_t
    c3 = c1 * 1.15                                        # faster: more time steps
    with ff.Plan(c1, dx, 0.5, angles) as P:
        G = _data(P, h, rng)
        P.reconstruct(G, 1e-3, 3)                         # captures both graphs
        for c in (c2, c3):
            nt_before = P.nt
            P.set_speed(c)
            with ff.Plan(c, dx, 0.5, angles) as Q:
                assert (P.nt, P.dt, P.cmax) == (Q.nt, Q.dt, Q.cmax)
                r_ref = Q.reconstruct(G, 1e-3, 3)
            r = P.reconstruct(G, 1e-3, 3)
            assert r.step == r_ref.step
            assert torch.equal(r.h, r_ref.h)
            assert np.array_equal(r.objective, r_ref.objective)
            if c is c3:
                assert P.nt > nt_before
        bad = c1.clone()
        bad[2, 2, 2] = -1.0
        nt = P.nt
        with pytest.raises(ff.FfpatError):
            P.set_speed(bad)
        assert P.nt == nt


def _trace(sizes, seed, n_iter=8, n_power=6, spacing=0.03):
    from paper_1901_06503_amd.serving import Job
    import paper_1901_06503_amd as ff
    jobs = []
    rng = np.random.default_rng(seed)
    t = 0.0
    for i, n in enumerate(sizes):
        dx, angles, c, h, r2 = _inputs(n, n, seed + i)
        with ff.Plan(c, dx, 0.5, angles) as P:
            G = _data(P, h, r2)
        torch.cuda.synchronize()
        jobs.append(Job(job_id=i, arrival=t, c=c.cpu().pin_memory(), G=G.cpu().pin_memory(), dx=dx, T=0.5,
                        angles=angles, lam=1e-3, n_iter=n_iter, n_power=n_power))
        t += float(rng.exponential(spacing))
    return jobs


def _clone(jobs):
    from paper_1901_06503_amd.serving import Job
    return [Job(job_id=j.job_id, arrival=j.arrival, c=j.c, G=j.G, dx=j.dx, T=j.T, angles=j.angles, lam=j.lam,
                n_iter=j.n_iter, n_power=j.n_power) for j in jobs]


def test_results_in_the_mix_equal_results_alone():
    from paper_1901_06503_amd.serving import Scheduler, run_serial, summary
    jobs = _trace([24, 40, 32, 48, 24, 40, 32, 24], 70)
    alone = run_serial(_clone(jobs))
    for policy in ("fill", "shortest", "all"):
        # two at a time even below the backlog, so that work really overlaps
        with Scheduler(hbm_budget=8 << 30, max_active=4, iters_per_turn=3, policy=policy,
                       low_concurrency=2) as sched:
            mixed = sched.run(_clone(jobs))
        assert sched.peak_running > 1                      # work really overlapped on the device
        assert sched.plans_reused > 0                      # later jobs ran on earlier jobs' plans
        for a, b in zip(sorted(alone, key=lambda j: j.job_id), sorted(mixed, key=lambda j: j.job_id)):
            assert a.status == b.status == "done"
            assert a.step == b.step
            assert torch.equal(a.h, b.h)
            assert np.array_equal(np.array(a.objective), np.array(b.objective))
        s = summary(mixed)
        assert s["jobs"] == len(jobs) and math.isfinite(s["latency_p99_s"])


def test_admission_respects_the_hbm_budget():
    from paper_1901_06503_amd.serving import Scheduler
    jobs = _trace([40, 40, 40, 40], 80, n_iter=4, n_power=3, spacing=0.0)
    one = jobs[0].footprint()
    with Scheduler(hbm_budget=int(1.5 * one), max_active=8) as sched:
        out = sched.run(jobs)
    assert all(j.status == "done" for j in out)
    assert sched.peak_active == 1 and sched.peak_bytes <= int(1.5 * one)
    assert sched.plans_created == 1 and sched.plans_reused == 3   # one plan serves all four
    with Scheduler(hbm_budget=int(2.5 * one), max_active=8) as sched2:
        sched2.run(_clone(jobs))
    assert sched2.peak_active == 2 and sched2.peak_bytes <= int(2.5 * one)
    # a job of another geometry makes an idle plan give way when the budget needs it
    other = _trace([40, 32], 81, n_iter=4, n_power=3, spacing=0.0)
    budget = jobs[0].footprint() + other[1].footprint() // 2
    with Scheduler(hbm_budget=budget, max_active=8) as sched3:
        out3 = sched3.run(_clone(jobs[:1]) + [other[1]])
    assert all(j.status == "done" for j in out3) and sched3.peak_bytes <= max(budget, other[1].footprint())


def test_failed_job_does_not_disturb_the_others():
    from paper_1901_06503_amd.serving import Scheduler, run_serial
    jobs = _trace([24, 32, 24], 90, n_iter=4, n_power=3)
    bad = _clone(jobs)
    bad[1].c = bad[1].c.clone()
    bad[1].c[3, 3, 3] = float("nan")                       # rejected at plan creation
    with Scheduler(hbm_budget=8 << 30, max_active=4) as sched:
        out = sched.run(bad)
    ref = run_serial(_clone(jobs))
    assert out[1].status.startswith("failed") and "FFPAT_EINVAL" in out[1].status
    for i in (0, 2):
        assert out[i].status == "done" and torch.equal(out[i].h, ref[i].h)

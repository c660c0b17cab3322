"""Serving loop: continuous batching of reconstruction jobs (Algorithm 8) on one GPU.

Each job carries its own grid, sound speed, angle set and data.  The loop
admits a job when it has arrived, a slot is free and its device footprint
(plan workspace + inputs + iterate, from ffpat_workspace_bytes) fits the
HBM budget; every admitted job gets its own stream and plan, its step size
from the power iteration, and then advances a few FB iterations per turn
(captured graphs replayed on its stream), so that the work of several jobs
overlaps on the device and late arrivals join between iterations of earlier
ones.  Finished jobs release their slot and memory.

`run_serial` is the plain baseline: one `ffpat_reconstruct` at a time in
arrival order.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    job_id: int
    arrival: float              # seconds after the start of the trace
    c: "object"                 # sound speed, device or pinned host tensor [nz][ny][nx]
    G: "object"                 # data [n_angles][nz][ns]
    dx: float
    T: float
    angles: np.ndarray
    lam: float = 1e-3
    n_iter: int = 50
    n_power: int = 20
    # results
    h: "object" = None
    step: float = float("nan")
    objective: list = field(default_factory=list)
    t_admit: float = float("nan")
    t_done: float = float("nan")
    status: str = "pending"

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival

    def footprint(self) -> int:
        from . import workspace_bytes
        esz = self.c.element_size()
        nvox = self.c.numel()
        return (workspace_bytes(tuple(self.c.shape), self.dx, self.T, self.angles,
                                dtype="float64" if esz == 8 else "float32")
                + (2 * nvox + self.G.numel()) * esz)


class _Active:
    def __init__(self, job, plan, stream, h, G):
        self.job, self.plan, self.stream, self.h, self.G = job, plan, stream, h, G
        self.done_iters = 0
        self.event = None
        self.busy = False
        self.bytes = 0
        self.last_chunk = 0


def _remaining_work(a) -> float:
    """Remaining point updates of an active job (two wave solves per FB iteration)."""
    return 2.0 * a.plan.nt * a.job.c.numel() * (a.job.n_iter - a.done_iters)


class Scheduler:
    """Continuous-batching scheduler.

    hbm_budget: device bytes the active jobs may hold together.
    max_active: slots.  iters_per_turn: FB iterations enqueued per job per turn.
    """

    def __init__(self, hbm_budget: int, max_active: int = 8, iters_per_turn: int = 5, concurrency: int = 0,
                 device="cuda"):
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.iters_per_turn = max(1, int(iters_per_turn))
        # how many admitted jobs advance at a time: 0 = all (round robin); k > 0 = the
        # oldest job plus the k - 1 with the least remaining work (the others stay
        # resident and wait)
        self.concurrency = int(concurrency)
        self.device = device
        self.peak_bytes = 0
        self.peak_active = 0
        self.peak_running = 0

    def _admit(self, job, now):
        import torch
        from . import Plan
        stream = torch.cuda.Stream(device=self.device)   # default priority
        with torch.cuda.stream(stream):
            c = job.c.to(self.device, non_blocking=True)
            G = job.G.to(self.device, non_blocking=True)
            h = torch.zeros(c.shape, dtype=c.dtype, device=self.device)
            plan = Plan(c, job.dx, job.T, job.angles, stream=stream)
            del c
            plan.fb_enqueue(G, job.lam, 0, h, step=0.0, n_power=job.n_power, stream=stream)
        a = _Active(job, plan, stream, h, G)
        a.event = torch.cuda.Event()
        a.event.record(stream)
        a.busy = True
        job.t_admit = now
        job.status = "running"
        return a

    def _advance(self, a):
        import torch
        j = a.job
        k = min(self.iters_per_turn, j.n_iter - a.done_iters)
        a.plan.fb_enqueue(a.G, j.lam, k, a.h, use_plan_step=True, stream=a.stream)
        a.done_iters += k
        a.last_chunk = k
        a.event = torch.cuda.Event()
        a.event.record(a.stream)
        a.busy = True

    def _collect(self, a):
        """Objective values of the chunk that just finished (stream already idle)."""
        step, obj = a.plan.fb_report(a.last_chunk, stream=a.stream)
        a.job.step = step
        a.job.objective.extend(obj.tolist())

    def run(self, jobs):
        """Serves `jobs` (arrival times in seconds from now) and returns them finished."""
        from . import FfpatError
        pending = sorted(jobs, key=lambda j: j.arrival)
        active: list[_Active] = []
        used = 0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            progressed = False
            # admission: arrived, a free slot, and the footprint fits
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                need = pending[0].footprint()
                if used + need > self.hbm_budget and active:
                    break
                job = pending.pop(0)
                try:
                    a = self._admit(job, now)
                except FfpatError as e:
                    job.status, job.t_done = f"failed: {e}", time.perf_counter() - t0
                    continue
                a.bytes = need
                used += need
                active.append(a)
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_active = max(self.peak_active, len(active))
                progressed = True
            # retire finished jobs; collect the objective of completed chunks
            for a in list(active):
                if a.busy and a.event.query():
                    a.busy = False
                    progressed = True
                    try:
                        if a.done_iters > 0:
                            self._collect(a)
                        if a.done_iters < a.job.n_iter:
                            continue
                        a.job.status = "done"
                    except FfpatError as e:
                        a.job.status = f"failed: {e}"
                    a.job.h = a.h
                    a.job.t_done = time.perf_counter() - t0
                    a.plan.close()
                    used -= a.bytes
                    active.remove(a)
            # advance: all idle jobs, or `concurrency` jobs: the oldest one (no job waits
            # for ever) plus those with the least remaining work (short jobs overtake)
            if self.concurrency > 0 and active:
                oldest = min(active, key=lambda a: a.job.arrival)
                rest = sorted((a for a in active if a is not oldest), key=_remaining_work)
                chosen = [oldest] + rest[:self.concurrency - 1]
            else:
                chosen = active
            for a in chosen:
                if not a.busy:
                    try:
                        self._advance(a)
                        progressed = True
                    except FfpatError as e:
                        a.job.status = f"failed: {e}"
                        a.job.t_done = time.perf_counter() - t0
                        a.plan.close()
                        used -= a.bytes
                        active.remove(a)
            self.peak_running = max(self.peak_running, sum(1 for a in active if a.busy))
            if not progressed:
                time.sleep(0.0002)
        return jobs


def run_serial(jobs, device="cuda"):
    """Plain baseline: jobs one at a time in arrival order with ffpat_reconstruct."""
    import torch
    from . import FfpatError, Plan
    t0 = time.perf_counter()
    for job in sorted(jobs, key=lambda j: j.arrival):
        while time.perf_counter() - t0 < job.arrival:
            time.sleep(0.0002)
        job.t_admit = time.perf_counter() - t0
        c = job.c.to(device)
        G = job.G.to(device)
        try:
            with Plan(c, job.dx, job.T, job.angles) as plan:
                res = plan.reconstruct(G, job.lam, job.n_iter, step=0.0, n_power=job.n_power)
            job.h, job.step, job.objective, job.status = res.h, res.step, res.objective.tolist(), "done"
        except FfpatError as e:
            job.status = f"failed: {e}"
        torch.cuda.synchronize()
        job.t_done = time.perf_counter() - t0
    return jobs


def summary(jobs):
    """jobs/s over the makespan and latency percentiles (arrival to result)."""
    done = [j for j in jobs if j.status == "done"]
    if not done:
        return {"jobs": 0}
    lat = np.array([j.latency for j in done])
    makespan = max(j.t_done for j in done) - min(j.arrival for j in jobs)
    return {"jobs": len(done), "failed": len(jobs) - len(done), "makespan_s": makespan,
            "jobs_per_s": len(done) / makespan, "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)), "latency_mean_s": float(lat.mean())}

"""Serving loop: continuous batching of reconstruction jobs (Algorithm 8) on one GPU.

Each job carries its own grid, sound speed, angle set and data.  The loop
admits a job when it has arrived, a slot is free and its device footprint
(plan workspace + inputs + iterate, from ffpat_workspace_bytes) fits the
HBM budget; every admitted job gets its own stream and plan.  A job's first
chunk of work is its power iteration (step size), then it advances a few FB
iterations per chunk (captured graphs replayed on its stream), so that the
work of several jobs overlaps on the device and late arrivals join between
iterations of earlier ones.  Which idle jobs get their next chunk is the
policy:

* "shortest" (default): the oldest job (so no job waits for ever) plus the
  `concurrency - 1` others that come first by remaining work in seconds minus
  `aging` times the time waited since arrival (short jobs overtake long ones,
  but only those that arrived less than a few of their remaining seconds
  earlier); `concurrency` applies while more than `backlog` jobs have arrived
  and are not finished; with fewer, `low_concurrency` (default 1: the oldest
  job, as the serial baseline runs it) joined by jobs of at most `join_voxels`
  grid points (default 128^3), up to `concurrency` in all: small grids, whose
  launches leave most of the device idle, need not wait behind a long job,
  which they slow only a little (sharing the device with larger jobs slows the
  long ones that set the tail).
* "fill": arrival order; the oldest job always runs, and later ones join
  while the running jobs hold at most `fill_voxels` grid points together
  (small grids, whose kernels leave most of the device idle, share it; a
  large grid runs alone at full speed).
* "all": every admitted job (round robin).

A finished job's plan, data buffer, iterate buffer and stream are kept for the
next job of the same geometry: ffpat_plan_set_speed gives the plan the new
sound speed and the captured iteration graphs are replayed as they are, so no
job after the first of its geometry allocates device memory, creates a plan or
captures a graph; kept plans give their memory back, least recently used
first, when an admission of another geometry needs it.  The result is copied
out of the kept iterate buffer on the job's stream.

What overlap can gain here is bounded: one job of the serial baseline is 98% or
more device time (plan creation, uploads, graph capture and destruction are 1-2%
of it: 64^3 41 ms, 128^3 128 ms, 192^3 318 ms, 256^3 1.04 s on MI355X), and the
multi-step stencil kernels of a 192^3 or 256^3 job hold every compute unit while
they run.  What remains is the 64^3 and 128^3 jobs, whose small launches leave the
device mostly idle, running in the gaps of the others.  On the 120-job trace
(grids 64^3..256^3, 50 iterations each, FP32), MI355X, "shortest" with concurrency
3, aging 4, backlog 5, small jobs (up to 128^3) joining below the backlog, chunks of
at least 20 ms: the device's capacity for this mix is about 3.7 jobs/s.  At 8 jobs/s
(saturated) 3.74 jobs/s against 3.51 serial (+6.5%; mean GPU activity 99.5% against
95.5%), median latency 8.0 s against 9.3 s, 99th percentile 14.4 s against 16.4 s.  At 4
jobs/s, near capacity, both finish with the arrivals (3.24 against 3.23 jobs/s) and the
gain is in latency: median 0.49 s against 1.15 s, 99th percentile 3.0 s against 3.7 s;
at 2 jobs/s median 0.306 s against 0.310 s, 99th percentile 1.63 s against 1.65 s.
Before the kernels of the 128^3..256^3 jobs got faster the device was further below
the 4 jobs/s of the trace (2.97 serial jobs/s, +8% for the scheduler).  Without the
joining rule the 2 jobs/s latencies were the serial baseline's; with any two jobs at a
time below the backlog the long jobs that set the tail slow down; run one at a time
always, the scheduler matches the serial baseline to 1%.

`run_serial` is the plain baseline: one `ffpat_reconstruct` at a time in
arrival order.
"""
from __future__ import annotations

import math
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


class _Slot:
    """A plan with its data, iterate and stream, kept for reuse by later jobs of the
    same geometry (grid, spacing, T, angles, precision): the workspace, the padded
    copies and the captured iteration graphs carry over; ffpat_plan_set_speed puts
    the next job's sound speed in."""

    def __init__(self, key, plan, G, h, stream, nbytes):
        self.key, self.plan, self.G, self.h, self.stream, self.bytes = key, plan, G, h, stream, nbytes
        self.last_used = 0.0


class _Active:
    def __init__(self, job, slot):
        self.job, self.slot = job, slot
        self.plan, self.stream, self.h, self.G = slot.plan, slot.stream, slot.h, slot.G
        self.done_iters = 0
        self.powered = False
        self.event = None
        self.busy = False
        self.last_chunk = 0


# Wave-operator rate that converts remaining point updates into seconds for the
# "shortest" policy's aging (the FP32 rate on MI355X is about 4e11 per second).
_POINT_UPDATES_PER_S = 4.0e11


def _remaining_work(a) -> float:
    """Remaining point updates of an active job (two wave solves per FB iteration or
    power step)."""
    left = a.job.n_iter - a.done_iters + (0 if a.powered else a.job.n_power)
    return 2.0 * a.plan.nt * a.job.c.numel() * left


def _geometry_key(job):
    c = job.c
    ang = np.ascontiguousarray(np.asarray(job.angles, dtype=np.float64))
    return (tuple(c.shape), str(c.dtype), float(job.dx), float(job.T), ang.tobytes(), tuple(job.G.shape))


class Scheduler:
    """Continuous-batching scheduler.

    hbm_budget: device bytes the jobs' plans, data and iterates may hold together
    (plans kept for reuse included: idle ones are released, least recently used
    first, when an admission needs their memory).
    max_active: slots.  iters_per_turn: FB iterations enqueued per job per turn, at least;
    more where fewer would take less than min_chunk_s seconds of device time (by the
    remaining-work estimate), so that small grids do not leave the device idle while
    the host enqueues their next chunk.
    policy: "fill", "shortest" or "all" (see the module docstring); fill_voxels is
    the fill threshold; concurrency the number of jobs "shortest" advances while more
    than `backlog` jobs have arrived and are not finished, low_concurrency otherwise
    (1: the oldest job alone, as the serial baseline would run it), joined, up to
    `concurrency` jobs, by jobs of at most `join_voxels` grid points; aging the seconds
    of waiting that offset a second of remaining work in "shortest".
    reuse_plans: keep finished jobs' plans for later jobs of the same geometry.
    """

    def __init__(self, hbm_budget: int, max_active: int = 8, iters_per_turn: int = 5, concurrency: int = 3,
                 policy: str = "shortest", fill_voxels: int = 192 ** 3, device="cuda", aging: float = 4.0,
                 reuse_plans: bool = True, backlog: int = 5, low_concurrency: int = 1, join_voxels: int = 128 ** 3,
                 min_chunk_s: float = 0.02):
        if policy not in ("fill", "shortest", "all"):
            raise ValueError(f"unknown policy {policy!r}")
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.iters_per_turn = max(1, int(iters_per_turn))
        self.min_chunk_s = float(min_chunk_s)
        self.policy = policy
        self.fill_voxels = int(fill_voxels)
        self.concurrency = max(1, int(concurrency))
        self.aging = float(aging)
        self.backlog = int(backlog)
        self.low_concurrency = max(1, int(low_concurrency))
        self.join_voxels = int(join_voxels)
        self.reuse_plans = bool(reuse_plans)
        self._waiting = 0
        self.device = device
        self.peak_bytes = 0
        self.peak_active = 0
        self.peak_running = 0
        self.plans_created = 0
        self.plans_reused = 0
        self._idle: list[_Slot] = []       # plans kept for reuse, not serving a job
        self._now = 0.0

    def _new_slot(self, job, key, need):
        import torch
        from . import Plan
        stream = torch.cuda.Stream(device=self.device)   # default priority
        with torch.cuda.stream(stream):
            c = job.c.to(self.device, non_blocking=True)
            G = job.G.to(self.device, non_blocking=True)
            h = torch.zeros(c.shape, dtype=c.dtype, device=self.device)
            plan = Plan(c, job.dx, job.T, job.angles, stream=stream)
            del c
        self.plans_created += 1
        return _Slot(key, plan, G, h, stream, need)

    def _reuse_slot(self, slot, job):
        import torch
        with torch.cuda.stream(slot.stream):
            c = job.c.to(self.device, non_blocking=True)
            slot.G.copy_(job.G, non_blocking=True)
            slot.h.zero_()
            slot.plan.set_speed(c, stream=slot.stream)
            del c
        self.plans_reused += 1
        return slot

    def _release(self, slot):
        slot.plan.close()

    def _admit(self, job, now, key, slot=None):
        slot = self._reuse_slot(slot, job) if slot is not None else self._new_slot(job, key, job.footprint())
        a = _Active(job, slot)
        job.t_admit = now
        job.status = "running"
        return a

    def _chunk(self, a):
        """FB iterations of an active job's next chunk: iters_per_turn, or more where those
        would take less than min_chunk_s of device time by the remaining-work estimate,
        never more than the job has left."""
        per_iter_s = 2.0 * a.plan.nt * a.job.c.numel() / _POINT_UPDATES_PER_S
        k = self.iters_per_turn
        if per_iter_s > 0:
            k = max(k, int(math.ceil(self.min_chunk_s / per_iter_s)))
        return min(k, a.job.n_iter - a.done_iters)

    def _advance(self, a):
        import torch
        j = a.job
        if not a.powered:                 # first chunk: the power iteration (step size)
            a.plan.fb_enqueue(a.G, j.lam, 0, a.h, step=0.0, n_power=j.n_power, stream=a.stream)
            a.powered = True
            k = 0
        else:
            k = self._chunk(a)
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

    def _finish(self, a, now):
        """Hands the iterate to the job (a copy on the job's stream, so that the slot's
        buffer can serve the next job) and keeps or releases the slot.  Returns an event
        recorded after the copy: the job is done when it has completed."""
        import torch
        with torch.cuda.stream(a.stream):
            a.job.h = a.h.clone()
        copied = torch.cuda.Event()
        copied.record(a.stream)
        a.slot.last_used = now
        if self.reuse_plans:
            self._idle.append(a.slot)
        else:
            self._release(a.slot)
        return copied

    def run(self, jobs):
        """Serves `jobs` (arrival times in seconds from now) and returns them finished."""
        import torch
        from . import FfpatError
        pending = sorted(jobs, key=lambda j: j.arrival)
        active: list[_Active] = []
        finishing = []                       # (job, event after its result's copy)
        t0 = time.perf_counter()

        def in_use():
            return sum(a.slot.bytes for a in active) + sum(s.bytes for s in self._idle)

        while pending or active or finishing:
            now = time.perf_counter() - t0
            self._now = now
            for jf in [f for f in finishing if f[1].query()]:
                jf[0].t_done = now
                finishing.remove(jf)
            self._waiting = len(active) + sum(1 for j in pending if j.arrival <= now)
            progressed = False
            # admission: arrived, a free slot, and the footprint fits (a kept plan of the
            # same geometry needs no new memory; idle kept plans give way when needed)
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                job = pending[0]
                key = _geometry_key(job)
                slot = next((s for s in self._idle if s.key == key), None)
                if slot is None:
                    need = job.footprint()
                    while self._idle and in_use() + need > self.hbm_budget:
                        victim = min(self._idle, key=lambda s: s.last_used)
                        self._idle.remove(victim)
                        self._release(victim)
                    if in_use() + need > self.hbm_budget and active:
                        break
                else:
                    self._idle.remove(slot)
                pending.pop(0)
                try:
                    a = self._admit(job, now, key, slot)
                except FfpatError as e:
                    job.status, job.t_done = f"failed: {e}", time.perf_counter() - t0
                    if slot is not None:
                        self._release(slot)
                    continue
                active.append(a)
                self.peak_bytes = max(self.peak_bytes, in_use())
                self.peak_active = max(self.peak_active, len(active))
                progressed = True
            # retire finished jobs; collect the objective of completed chunks
            for a in list(active):
                if a.busy and a.event.query():
                    a.busy = False
                    progressed = True
                    try:
                        if a.last_chunk > 0:
                            self._collect(a)
                        if a.done_iters < a.job.n_iter:
                            continue
                        a.job.status = "done"
                    except FfpatError as e:
                        a.job.status = f"failed: {e}"
                    finishing.append((a.job, self._finish(a, time.perf_counter() - t0)))
                    active.remove(a)
            chosen = self._choose(active)
            for a in chosen:
                if not a.busy:
                    try:
                        self._advance(a)
                        progressed = True
                    except FfpatError as e:
                        a.job.status = f"failed: {e}"
                        a.job.t_done = time.perf_counter() - t0
                        self._release(a.slot)
                        active.remove(a)
            self.peak_running = max(self.peak_running, sum(1 for a in active if a.busy))
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize(self.device)        # results copied out on the jobs' streams
        return jobs

    def close(self):
        """Releases the plans kept for reuse."""
        for s in self._idle:
            self._release(s)
        self._idle = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _choose(self, active):
        """The admitted jobs that may start their next chunk now (see the policies)."""
        if not active or self.policy == "all":
            return active
        order = sorted(active, key=lambda a: (a.job.arrival, a.job.job_id))
        if self.policy == "shortest":
            now = self._now
            prio = lambda a: (_remaining_work(a) / _POINT_UPDATES_PER_S - self.aging * (now - a.job.arrival),
                              a.job.arrival, a.job.job_id)
            rest = sorted(order[1:], key=prio)
            if self._waiting > self.backlog:
                return [order[0]] + rest[:self.concurrency - 1]
            conc = min(self.low_concurrency, self.concurrency)
            small = [a for a in rest[conc - 1:] if a.job.c.numel() <= self.join_voxels]
            return [order[0]] + rest[:conc - 1] + small[:self.concurrency - conc]
        chosen, vox = [order[0]], order[0].job.c.numel()
        for a in order[1:]:
            if vox + a.job.c.numel() > self.fill_voxels:
                break
            chosen.append(a)
            vox += a.job.c.numel()
        return chosen


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

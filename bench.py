"""Benchmark of the one-step full-field PAT hot path on one MI355X.

A step is one iteration of Algorithm 8 (forward wave solve, projection,
residual + ramp filter + FP64 objective, backprojection, adjoint wave solve,
prox update) on the 256^3 workload: 256 angles, T = 0.5, FP32 fields with
FP64 reductions, seeded synthetic phantom (balls + vessel-like tubes) and
sound speed (5 Gaussian bumps clamped to [0.8, 1.2]).  The step size comes
from a 20-step power iteration done before the timed region.

Prints one JSON line.  See --help.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "wave-op Gpt-updates/s; FB iter/s at 256³ FP32 vs FP64; recon p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--recipe", default="c256", help="synthetic workload recipe (c128, c256, c384)")
    ap.add_argument("--dtype", default="float32", choices=["float32", "float64"])
    ap.add_argument("--fp64-compare", type=int, default=1, help="also time FB iterations in FP64 (1/0)")
    ap.add_argument("--reg", default="l2", choices=["l2", "grad"],
                    help="regulariser of the timed FB iterations: l2 (prox in closed form) or grad "
                         "(R = 1/2 ||D h||^2, prox by conjugate gradients on the device)")
    ap.add_argument("--cpu-baseline", type=int, default=1, help="time the oracle on a bounded sample (1/0)")
    ap.add_argument("--naive-stencil", action="store_true")
    ap.add_argument("--n", type=int, default=0, help="--mode wave: grid edge instead of the recipe's")
    ap.add_argument("--nz", type=int, default=0, help="--mode wave: planes (default: the grid edge)")
    ap.add_argument("--stencil", default="auto", choices=["auto", "single", "pairs", "triples"],
                    help="--mode wave: leapfrog steps per stencil pass (auto: the plan's choice)")
    ap.add_argument("--seed", type=int, default=3001)
    ap.add_argument("--blocks", type=int, default=0,
                    help="--mode stream: work-groups per launch (0: the best of 2048, 4096, 8192, 16384)")
    ap.add_argument("--mode", default="fb", choices=["fb", "wave", "copy", "stream", "serve", "precision", "paper2d"],
                    help="fb: the benchmark; wave: only W_T applications (for counter runs); "
                         "copy: a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--reps", type=int, default=2, help="applications in --mode wave / copies in --mode copy")
    ap.add_argument("--jobs", type=int, default=120, help="--mode serve: jobs in the trace")
    ap.add_argument("--rate", type=float, default=4.0, help="--mode serve: mean arrivals per second (Poisson)")
    ap.add_argument("--iters", type=int, default=None,
                    help="--mode serve: FB iterations per job (50); --mode precision: iterations (200)")
    ap.add_argument("--slots", type=int, default=6, help="--mode serve: admitted (resident) jobs")
    ap.add_argument("--policy", default="shortest", choices=["fill", "shortest", "all"],
                    help="--mode serve: scheduler policy (shortest: the oldest job + the least remaining work; "
                         "fill: arrival order, small grids share the device)")
    ap.add_argument("--fill-voxels", type=int, default=192 ** 3,
                    help="--mode serve, policy fill: grid points the running jobs may hold together")
    ap.add_argument("--concurrency", type=int, default=3,
                    help="--mode serve, policy shortest: jobs advancing at a time")
    ap.add_argument("--serial", type=int, default=1, help="--mode serve: also run the serial baseline (1/0)")
    ap.add_argument("--aging", type=float, default=4.0,
                    help="--mode serve, policy shortest: seconds of waiting that offset a second of remaining work")
    ap.add_argument("--low-concurrency", type=int, default=1,
                    help="--mode serve, policy shortest: jobs advanced together while at most --backlog are waiting")
    ap.add_argument("--backlog", type=int, default=5,
                    help="--mode serve, policy shortest: jobs in the system above which --concurrency applies")
    ap.add_argument("--join-voxels", type=int, default=128 ** 3,
                    help="--mode serve and the serving leg, policy shortest: below --backlog, jobs of at most "
                         "this many grid points run beside the oldest (0: none)")
    ap.add_argument("--serve-jobs", type=int, default=120,
                    help="--mode fb: jobs in the serving leg (the 120-job trace at 4 jobs/s: p50/p99 latency, "
                         "jobs/s against the serial baseline); 0 skips it")
    ap.add_argument("--serve-saturated-jobs", type=int, default=60,
                    help="--mode fb: jobs of a second serving trace at 8 jobs/s, above the device's capacity for "
                         "the mix (throughput of the served form against the serial baseline when both are "
                         "device-bound); 0 skips it, and so does --serve-jobs 0")
    ap.add_argument("--operator-384", type=int, default=1,
                    help="--mode fb: also time the forward operator A = X W_T at 384^3 / 360 angles / T = 0.6 "
                         "in FP32 and FP64 (the operator HBM fraction, 1/0)")
    return ap.parse_args()


def run_precision(args):
    """384^3 / 360 angles / T = 0.6: Algorithm 8 for --iters iterations (default 200) in
    FP32 fields with FP64 reductions and in all-FP64, on the same data; reports the
    relative L2 difference of the two reconstructions and each one's error against
    the phantom, and the FB iteration rate of both.  Also the operator HBM fraction of
    the forward operator A = X W_T: (w N^3 n_t + w N^3 + w N_phi N^2) / t_A / 8 TB/s with
    w = 4 words of the field type per leapfrog point update (16 B FP32, 32 B FP64) and
    one word per voxel and per bin for the projection, t_A from HIP events."""
    import numpy as np
    import torch
    import paper_1901_06503_amd as ff
    import synth
    case = synth.make_case("c384", args.seed)
    case.c = case.c.astype(np.float32).astype(np.float64)         # identical c (and n_t) in both plans
    case.h_true = case.h_true.astype(np.float32).astype(np.float64)
    n_iter = args.iters if args.iters is not None else case.n_iter
    dev = torch.device("cuda:0")
    out = {"mode": "precision", "grid": case.n, "angles": len(case.angles), "T": case.T, "iters": n_iter}
    recon = {}
    with ff.Plan(torch.from_numpy(case.c).to(dev), case.dx, case.T, case.angles) as P64:
        clean = P64.forward(torch.from_numpy(case.h_true).to(dev))
        G64 = clean + case.noise_level * float(clean.mean()) * torch.from_numpy(case.noise).to(dev)
        out["nt"] = P64.nt
    for name, dtype in (("f32", torch.float32), ("f64", torch.float64)):
        with ff.Plan(torch.from_numpy(case.c).to(dev, dtype), case.dx, case.T, case.angles) as P:
            G = G64.to(dtype)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = P.reconstruct(G, case.lam, n_iter, step=0.0, n_power=case.n_power)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            recon[name] = res.h.double()
            out[name] = {"seconds": t, "fb_iter_per_s_incl_power": n_iter / t, "step": res.step,
                         "objective_first": float(res.objective[0]), "objective_last": float(res.objective[-1]),
                         "steps_per_pass": P.steps_per_pass}
            x = res.h.clone()
            g = P.forward(x)
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(3):
                P.forward(x, out=g, stream=stream)
            e1.record(stream)
            e1.synchronize()
            t_a = e0.elapsed_time(e1) / 1e3 / 3
            esz = 4 if dtype == torch.float32 else 8
            n3, nang = case.n ** 3, len(case.angles)
            alg = esz * (4 * n3 * P.nt + n3 + nang * case.n ** 2)
            out[name].update(forward_ms=1e3 * t_a, forward_gpt_updates_per_s=n3 * P.nt / t_a / 1e9,
                             operator_hbm_frac=alg / t_a / (HBM_PEAK_GBS * 1e9))
            log(f"{name}: {t:.1f}s for {n_iter} iterations + {case.n_power} power steps")
    h_true = torch.from_numpy(case.h_true).to(dev)
    d = float((recon["f32"] - recon["f64"]).norm() / recon["f64"].norm())
    out["rel_l2_f32_vs_f64"] = d
    for name in ("f32", "f64"):
        out[name]["rel_l2_vs_phantom"] = float((recon[name] - h_true).norm() / h_true.norm())
    print(json.dumps(out), flush=True)


def run_paper2d(args):
    """The paper's 2D experiment geometry (Sec. 4.1/4.2) on synthetic inputs: one-step
    (Algorithm 8) vs two-step (Algorithm 9) vs one-step with the mean constant speed,
    R = 1/2 ||grad h||^2, 60 iterations, 20% noise, stripe [-1, 1] missing, for a sweep
    of lambda (the paper's lambda = 0.5 and s = 0.2 belong to its own, unstated,
    discrete normalisation; the step here comes from the power iteration)."""
    import numpy as np
    import torch
    import paper_1901_06503_amd as ff
    import synth
    k = synth.paper2d_case(args.seed)
    dev = torch.device("cuda:0")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    n_iter = args.iters or 60
    lams = [0.5, 5e-2, 5e-3, 5e-4, 5e-5]
    out = {"mode": "paper2d", "grid": k["h"].shape[-1], "angles": len(k["angles"]), "T": k["T"], "iters": n_iter,
           "regulariser": "1/2 ||grad h||^2", "noise": "20% of mean(XWh)", "missing_stripe": k["stripe"],
           "runs": []}
    h_true = f32(k["h"])
    support = torch.from_numpy(k["support"]).to(dev)
    rel = lambda h: float((h - h_true).norm() / h_true.norm())
    cmean = float(np.mean(k["c"]))
    with ff.Plan(f32(k["c"]), k["dx"], k["T"], k["angles"], ndim=2) as P, \
            ff.Plan(torch.full_like(f32(k["c"]), cmean), k["dx"], k["T"], k["angles"], ndim=2) as Pc:
        out["nt"] = P.nt
        mask = P.stripe_mask(k["stripe"])
        clean = P.forward(h_true)
        noise = f32(k["noise"]) * 0.2 * float(clean.double().mean())
        out["data_error"] = float(noise.norm() / clean.norm())
        G = (clean + noise) * mask
        g = P.fbp(G)
        for lam in lams:
            t0 = time.perf_counter()
            one = P.reconstruct(G, lam, n_iter, reg="grad", positivity=False, det_mask=mask, support=support,
                                cg_maxit=400)
            t_one = time.perf_counter() - t0
            two = P.reconstruct(g, lam, n_iter, reg="grad", positivity=False, two_step=True, support=support,
                                cg_maxit=400)
            const = Pc.reconstruct(G, lam, n_iter, reg="grad", positivity=False, det_mask=mask,
                                   support=support, cg_maxit=400)
            run = {"lambda": lam, "one_step_rel_error": rel(one.h), "two_step_rel_error": rel(two.h),
                   "constant_speed_rel_error": rel(const.h), "one_step_seconds": t_one, "step": one.step}
            out["runs"].append(run)
            log(f"paper2d {run}")
    best = min(out["runs"], key=lambda r: r["one_step_rel_error"])
    out["best_lambda"] = best["lambda"]
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving workload: Poisson arrivals, grids uniform over {64,128,192,256}^3,
    angles = grid edge, 50 FB iterations + 20 power steps each, FP32.  Runs the
    same trace through the serial baseline and the continuous-batching scheduler."""
    print(json.dumps(serve_summary(args.jobs, args.rate, args.iters or 50, args.slots, args.concurrency,
                                   args.policy, args.fill_voxels, args.serial, args.seed, args.aging,
                                   args.low_concurrency, args.backlog, args.join_voxels)), flush=True)


class BusySampler:
    """Mean GPU activity (percent of time the graphics engine was busy, as the driver
    reports it through torch.cuda.utilization) sampled every `period` seconds while
    the block runs; None where the query is not available."""

    def __init__(self, torch, period=0.1):
        import threading
        self.torch, self.period, self.samples = torch, period, []
        self._stop = threading.Event()
        self._thread = threading.Thread(target=self._run, daemon=True)

    def _run(self):
        while not self._stop.is_set():
            try:
                self.samples.append(float(self.torch.cuda.utilization()))
            except Exception:             # no activity query on this system
                return
            self._stop.wait(self.period)

    def __enter__(self):
        self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._thread.join()

    @property
    def mean(self):
        return sum(self.samples) / len(self.samples) if self.samples else None


def serve_summary(n_jobs, rate, iters, slots, concurrency, policy, fill_voxels, serial, seed, aging=1.0,
                  low_concurrency=1, backlog=5, join_voxels=128 ** 3):
    import numpy as np
    import torch
    import paper_1901_06503_amd as ff
    from paper_1901_06503_amd import serving
    import synth
    rng = np.random.default_rng(seed)
    sizes = rng.choice([64, 128, 192, 256], size=n_jobs)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for i, (n, t) in enumerate(zip(sizes, arrivals)):
        dx, angles, c, h = synth.torch_case(int(n), int(n), seed * 1000 + i)
        with ff.Plan(c, dx, 0.5, angles) as P:
            g = P.forward(h)
            noise = torch.from_numpy(rng.standard_normal(P.data_shape)).to(g.device, g.dtype)
            G = g + 0.02 * float(g.double().mean()) * noise
        torch.cuda.synchronize()
        jobs.append(serving.Job(job_id=i, arrival=float(t), c=c.cpu().pin_memory(), G=G.cpu().pin_memory(), dx=dx,
                                T=0.5, angles=angles, lam=1e-3, n_iter=iters, n_power=20))
        if (i + 1) % 20 == 0:
            log(f"trace: {i + 1}/{n_jobs} jobs generated")
    clone = lambda: [serving.Job(job_id=j.job_id, arrival=j.arrival, c=j.c, G=j.G, dx=j.dx, T=j.T,
                                 angles=j.angles, lam=j.lam, n_iter=j.n_iter, n_power=j.n_power) for j in jobs]
    base = None
    if serial:
        log("serial baseline")
        with BusySampler(torch) as busy:
            base = serving.summary(serving.run_serial(clone()))
        base["gpu_busy_mean_pct"] = busy.mean
        log(f"serial: {base}")
    free, total = torch.cuda.mem_get_info()
    log("continuous batching")
    with serving.Scheduler(hbm_budget=int(0.5 * free), max_active=slots, iters_per_turn=5,
                           concurrency=concurrency, policy=policy, fill_voxels=fill_voxels, aging=aging,
                           low_concurrency=low_concurrency, backlog=backlog, join_voxels=join_voxels) as sched:
        with BusySampler(torch) as busy:
            mixed_jobs = sched.run(clone())
    mixed = serving.summary(mixed_jobs)
    mixed["gpu_busy_mean_pct"] = busy.mean
    log(f"scheduler: {mixed}")
    return {"mode": "serve", "jobs": n_jobs, "rate_per_s": rate, "iters": iters, "slots": slots, "policy": policy,
            "fill_voxels": fill_voxels, "concurrency": concurrency, "aging": aging,
            "low_concurrency": low_concurrency, "backlog": backlog, "join_voxels": join_voxels, "serial": base,
            "continuous_batching": mixed,
            "peak_active": sched.peak_active, "peak_running": sched.peak_running, "peak_bytes": sched.peak_bytes,
            "plans_created": sched.plans_created, "plans_reused": sched.plans_reused,
            "throughput_gain": mixed["jobs_per_s"] / base["jobs_per_s"] if base else None}


def run_wave_only(args):
    """Applies W_T `reps` times on the workload (n_t leapfrog launches each) and exits."""
    import torch
    import paper_1901_06503_amd as ff
    import synth
    import numpy as np
    dtype = torch.float32 if args.dtype == "float32" else torch.float64
    r = synth.RECIPES[args.recipe]
    n = args.n or r["n"]
    nz = args.nz or n
    dx = synth.grid_spacing(n)
    c = synth.sound_speed((nz, n, n), dx, np.random.default_rng(args.seed), r["bumps"], r["amp"], r["clamp"])
    plan = ff.Plan(torch.from_numpy(c).to("cuda", dtype), dx, r["T"], synth.uniform_angles(r["n_angles"]),
                   naive_stencil=args.naive_stencil,
                   stencil_steps={"auto": None, "single": 1, "pairs": 2, "triples": 3}[args.stencil])
    h = torch.randn((nz, n, n), dtype=dtype, device="cuda")
    out = torch.empty_like(h)
    plan.wave(h, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(args.reps):
        plan.wave(h, out=out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / (args.reps * plan.nt)
    env = {k: v for k, v in os.environ.items() if k.startswith("FFPAT_")}
    print(json.dumps({"mode": "wave", "n": n, "nz": nz, "dtype": args.dtype, "nt": plan.nt, "reps": args.reps,
                      "steps_per_pass": plan.steps_per_pass, "stencil_shape": list(plan.stencil_shape),
                      "us_per_step": us, "gpt_updates_per_s": nz * n * n / us / 1e3, "env": env}), flush=True)


def run_copy_only(args):
    """Copies a 1 GiB buffer `reps` times (1 GiB read + 1 GiB written per copy)."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for r in range(args.reps):
        b.copy_(a)
    e1.record(stream)
    e1.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / args.reps
    log(f"{args.reps} copies done")
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                      "reps": args.reps, "GBps_read_plus_write": 8 * n / s / 1e9}))


def probe_library():
    """libffpat_probe.so (streaming-ceiling kernels), or None if it is not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_1901_06503_amd", "libffpat_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.ffpat_probe_stream.restype = ctypes.c_int
    lib.ffpat_probe_stream.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_size_t, ctypes.c_int,
                                                                              ctypes.c_void_p]
    return lib


def probe_stream_us(torch, lib, pattern, fields, blocks, reps):
    """Average duration (us, HIP events on the current stream) of `reps` launches of a
    streaming pattern over `fields` (five FP32 tensors of one size), rotating the fields
    so that each launch reads what the previous one wrote."""
    import ctypes
    stream = torch.cuda.current_stream()
    count = fields[0].numel()

    def launch(r):
        if pattern == 0:
            ptrs = [fields[(r + i) % 5].data_ptr() for i in range(5)]
        else:
            ptrs = [fields[r % 2].data_ptr(), None, None, fields[(r + 1) % 2].data_ptr(), None]
        rc = lib.ffpat_probe_stream(pattern, *ptrs, count, blocks, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"ffpat_probe_stream returned {rc}")

    for r in range(3):
        launch(r)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for r in range(reps):
        launch(r)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def run_stream(args):
    """Streaming ceilings (libffpat_probe.so): the two-step stencil's streams (three
    fields read, two written) and a copy, over FP32 fields of n^3 points (256 and 384,
    or --n), rotating the five fields so that each launch reads what the previous one
    wrote, as the leapfrog does.  The best of four launch widths per pattern and size
    (or --blocks).  --dtype float64: fields of the same bytes as n^3 FP64 points."""
    import torch
    lib = probe_library()
    if lib is None:
        raise SystemExit("libffpat_probe.so is missing: build it with `python -m paper_1901_06503_amd.build`")
    reps = max(args.reps, 10)
    words_per_point = 2 if args.dtype == "float64" else 1
    for n in ([args.n] if args.n else [256, 384]):
        count = n ** 3 * words_per_point
        f = [torch.zeros(count, dtype=torch.float32, device="cuda") for _ in range(5)]
        out = {"mode": "stream", "n": n, "dtype": args.dtype, "bytes_per_field": 4 * count, "reps": reps}
        for pattern, name, words in ((0, "read3_write2", 5), (1, "read1_write1", 2)):
            best = None
            for blocks in ([args.blocks] if args.blocks > 0 else [2048, 4096, 8192, 16384]):
                us = probe_stream_us(torch, lib, pattern, f, blocks, reps)
                if best is None or us < best[0]:
                    best = (us, blocks)
            out[name] = {"us_per_launch": best[0], "blocks": best[1],
                         "TBps": words * 4 * count / (best[0] * 1e-6) / 1e12}
            log(f"stream n={n} {name}: {best[0]:.2f} us, {out[name]['TBps']:.3f} TB/s")
        print(json.dumps(out))
        del f
        torch.cuda.empty_cache()


def stream_ceiling(torch, bytes_per_launch, achieved):
    """The two-step stencil's streams at the workload's field size (three fields read,
    two written, bytes_per_launch in all) in a plain streaming kernel: what a kernel
    with these streams can reach on this device, and the stencil's share of it."""
    lib = probe_library()
    if lib is None:
        return None
    count = bytes_per_launch // 5 // 4
    f = [torch.zeros(count, dtype=torch.float32, device="cuda") for _ in range(5)]
    us, blocks = min((probe_stream_us(torch, lib, 0, f, b, 20), b) for b in (8192, 16384))
    del f
    torch.cuda.empty_cache()
    gbps = bytes_per_launch / (us * 1e-6) / 1e9
    return {"kernel": "read3_write2", "achieved": gbps, "unit": "GB/s", "us_per_launch": us, "blocks": blocks,
            "frac": achieved / gbps}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(args, torch, ff, synth, dtype):
    case = synth.make_case(args.recipe, args.seed)
    dev = torch.device("cuda:0")
    c = torch.from_numpy(case.c).to(dev, dtype)
    plan = ff.Plan(c, case.dx, case.T, case.angles, naive_stencil=args.naive_stencil)
    h_true = torch.from_numpy(case.h_true).to(dev, dtype)
    clean = plan.forward(h_true)
    sigma = case.noise_level * float(clean.double().mean())
    G = clean + sigma * torch.from_numpy(case.noise).to(dev, dtype)
    torch.cuda.synchronize()
    return case, plan, G


def time_fb(torch, plan, G, lam, steps, warmup, reg="l2"):
    h = torch.zeros(plan.shape, dtype=plan.dtype, device=G.device)
    pos = reg == "l2"                  # the gradient prox has no positivity constraint
    t0 = time.perf_counter()
    res = plan.reconstruct(G, lam, 0, step=0.0, n_power=20, h0=h, reg=reg, positivity=pos)   # power iteration
    torch.cuda.synchronize()
    t_power = time.perf_counter() - t0
    if warmup:
        plan.reconstruct(G, lam, warmup, h0=h, use_plan_step=True, reg=reg, positivity=pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = plan.reconstruct(G, lam, steps, h0=h, use_plan_step=True, reg=reg, positivity=pos)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return t, t_power, out


def time_wave(torch, plan, reps=3):
    """Seconds per W_T application, from HIP events around back-to-back
    applications on the stream the kernels are launched on."""
    x = torch.randn(plan.shape, dtype=plan.dtype, device="cuda")
    y = torch.empty_like(x)
    plan.wave(x, out=y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.wave(x, out=y, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def stencil_roofline(torch, ff, plan, c, dx, T, angles, dtype):
    """The dominant kernel of the path (the leapfrog stencil) and its average launch
    duration, measured live.  A forward W_T solve is n_t leapfrog steps: with one step
    per pass, n_t launches of wave_step_blocked; with two steps per pass in
    wave_step2_split, M = 1 + (n_t - 2) // 2 launches of it (the first starts the solve
    from p(0)) and a single step for an odd remainder, in the other two-step kernel one
    first-step launch, M = (n_t - 1) // 2 two-step launches and a single step for an
    odd remainder; with three, M = 1 + (n_t - 3) // 3 three-step launches
    (the first starts the solve from p(0)) and a single step or a pair for the
    remaining (n_t - 3) % 3 steps.  The k-step kernel's duration is
    (t(W_T) - t_first - t_rest) / M, with the single-step duration measured on a plan
    that runs one step per pass and the pair duration, where needed, derived the same
    way on a two-step plan.
    Bytes per launch, two ways: algorithmic = 4 words per point update (read p(k),
    p(k-1), k'; write p(k+1): 16 B FP32, 32 B FP64) x the updates a launch makes per
    voxel (1, 2 or 3); compulsory = the words per voxel a launch must move at least
    (4 for one step; read p(k-1), p(k), k', write the last two levels: 5 for two or
    three steps)."""
    esz = 4 if dtype == torch.float32 else 8
    f64 = dtype == torch.float64
    nvox = math.prod(plan.shape)
    t_w = time_wave(torch, plan)
    k = plan.steps_per_pass
    out = {"t_wave": t_w, "steps_per_pass": k}
    if k == 1:
        out.update(kernel="wave_step_blocked", t_launch=t_w / plan.nt, alg_bytes=4 * esz * nvox,
                   compulsory_bytes=4 * esz * nvox, updates_per_launch=1)
        return out
    with ff.Plan(c, dx, T, angles, stencil_steps=1) as ps:
        t_single = time_wave(torch, ps) / ps.nt
    t_pair = None
    if k == 3:
        with ff.Plan(c, dx, T, angles, stencil_steps=2) as p2:
            t_w2 = time_wave(torch, p2)
            if multi_kernel_name(p2, f64) == "wave_step2_split" and p2.nt >= 2:
                pairs2, singles2 = divmod(p2.nt - 2, 2)      # the first pass is a pair too
                pairs2 += 1
                t_pair = (t_w2 - singles2 * t_single) / pairs2
            else:
                pairs2, singles2 = divmod(p2.nt - 1, 2)
                t_pair = (t_w2 - (1 + singles2) * t_single) / pairs2
    if k == 3 and plan.nt >= 3:
        # the solve's first pass is a three-step launch too (it starts from p(0))
        full, rest = divmod(plan.nt - 3, 3)
        full, t_first = full + 1, 0.0
    elif k == 2 and plan.nt >= 2 and multi_kernel_name(plan, f64) == "wave_step2_split":
        # wave_step2_split starts the solve from p(0) as well
        full, rest = divmod(plan.nt - 2, 2)
        full, t_first = full + 1, 0.0
    else:
        (full, rest), t_first = divmod(plan.nt - 1, k), t_single
    if full == 0:                       # too few steps for a multi-step launch
        out.update(kernel="wave_step_blocked", t_launch=t_single, alg_bytes=4 * esz * nvox,
                   compulsory_bytes=4 * esz * nvox, updates_per_launch=1)
        return out
    t_rest = 0.0 if rest == 0 else (t_single if rest == 1 else t_pair)
    out.update(kernel=multi_kernel_name(plan, f64), t_launch=(t_w - t_first - t_rest) / full,
               alg_bytes=k * 4 * esz * nvox, compulsory_bytes=5 * esz * nvox, updates_per_launch=k,
               t_single_launch=t_single)
    if t_pair is not None:
        out["t_pair_launch"] = t_pair
    return out


def multi_kernel_name(plan, f64):
    """The kernel a plan's multi-step launches run: for three steps per pass
    wave_step3_wide (FP32, pairs of x-adjacent points, 1024 threads) or
    wave_step3_split (FP64); for two, wave_step2_split with 8-byte elements and the
    64 x 16 element tile (FP64, and FP32 as pairs of points, a 128-point-wide tile on
    a grid of even nx), else wave_step2_blocked."""
    if plan.steps_per_pass == 3:
        return "wave_step3_split" if f64 else "wave_step3_wide"
    if os.environ.get("FFPAT_STENCIL2_SPLIT", "1") == "0":
        return "wave_step2_blocked"
    tx, ty, _ = plan.stencil_shape
    if f64:
        return "wave_step2_split" if (tx, ty) == (64, 16) else "wave_step2_blocked"
    return "wave_step2_split" if tx == 128 and plan.shape[2] % 2 == 0 else "wave_step2_blocked"


def operator_384(torch, ff, synth, seed):
    """The forward operator A = X W_T at the precision workload's shape (384^3, 360
    angles, T = 0.6, c with 10 bumps clamped to [0.75, 1.25]), where each field
    (226 MB FP32) exceeds the 256 MB MALL with the others: the operator HBM fraction
    (w N^3 n_t + w N^3 + w N_phi N^2) / t_A / 8 TB/s, w = 4 words of the field type
    per point update and one per voxel and per bin for the projection, t_A from HIP
    events around back-to-back applications, in FP32 and FP64; and the multi-step
    launch's duration and algorithmic rate there."""
    out = {"workload": "384^3 grid, 360 angles, T=0.6, c in [0.75, 1.25] (10 bumps)"}
    n, nang = 384, 360
    for name, dtype in (("f32", torch.float32), ("f64", torch.float64)):
        dx, angles, c, h = synth.torch_case(n, nang, seed, dtype=dtype, n_bumps=10, amp=0.2, clamp=(0.75, 1.25))
        with ff.Plan(c, dx, 0.6, angles) as P:
            g = P.forward(h)
            stream = torch.cuda.current_stream()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                P.forward(h, out=g, stream=stream)
            e1.record(stream)
            e1.synchronize()
            t_a = e0.elapsed_time(e1) / 1e3 / 3
            esz = 4 if dtype == torch.float32 else 8
            n3 = n ** 3
            alg = esz * (4 * n3 * P.nt + n3 + nang * n * n)
            roof = stencil_roofline(torch, ff, P, c, dx, 0.6, angles, dtype)
            out[name] = {"nt": P.nt, "forward_ms": 1e3 * t_a, "operator_hbm_frac": alg / t_a / (HBM_PEAK_GBS * 1e9),
                         "kernel": roof["kernel"], "avg_launch_us": roof["t_launch"] * 1e6,
                         "achieved_GBps": roof["alg_bytes"] / roof["t_launch"] / 1e9,
                         "frac": roof["alg_bytes"] / roof["t_launch"] / 1e9 / HBM_PEAK_GBS,
                         "frac_compulsory": roof["compulsory_bytes"] / roof["t_launch"] / 1e9 / HBM_PEAK_GBS}
        del c, h, g
        torch.cuda.empty_cache()
        log(f"384^3 {name}: {out[name]}")
    return out


def host_cpu_model():
    """The host CPU as /proc/cpuinfo names it, with its family and model numbers (a
    virtual machine may report only a generic name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model") and k not in info:
                    info[k] = v
            if len(info) == 3:
                break
    except OSError:
        pass
    if "model name" not in info:
        import platform
        return platform.processor() or "unknown"
    extra = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model") if k in info)
    return info["model name"] + (f" ({extra})" if extra else "")


def cpu_baseline(case, G, step):
    """The oracle (FP64 C, OpenMP) timed on one full Algorithm-8 iteration of the same
    workload: same c, same G, same step size, h_0 = 0."""
    import numpy as np
    import oracle
    n = case.n
    g = oracle.Geometry(nx=n, ny=n, nz=n, dx=case.dx, T=case.T, angles=case.angles)
    G_np = G.double().cpu().numpy()
    t0 = time.perf_counter()
    oracle.fb(g, case.c, G_np, case.lam, step=step, n_iter=1, flags=oracle.POSITIVITY | oracle.PRECOND)
    t = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the oracle's own wave-solve rate, on a bounded sample: one W_T of the 128^3 grid
    # (same dx rule, T and sound-speed recipe)
    import synth
    small = synth.make_case("c128", 2001)
    gs = oracle.Geometry(nx=small.n, ny=small.n, nz=small.n, dx=small.dx, T=small.T, angles=small.angles)
    nt_small = oracle.plan_info(gs, small.c)[0]
    t1 = time.perf_counter()
    oracle.wave(gs, small.c, small.h_true)
    tw = time.perf_counter() - t1
    return {"value": 1.0 / t, "unit": "FB iter/s", "cores": cores, "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": f"one full FB iteration of the {n}^3 / {len(case.angles)}-angle workload in FP64 "
                      f"({t:.1f} s: 2 wave solves, X, Lambda, X^T, prox)",
            "oracle_wave_gpt_updates_per_s": small.n ** 3 * nt_small / tw / 1e9,
            "oracle_wave_sample": f"one W_T of the 128^3 grid, n_t = {nt_small} ({tw:.2f} s)"}


def stored_traffic(kernel, recipe, dtype_name):
    """HBM bytes per launch of `kernel` from the committed counter runs, if the
    stencil source is unchanged since they were taken (else None)."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1901_06503_amd", "csrc", "kernels_wave.hip")
    note = os.path.join(ROOT, "profiles", "wave_step_hbm_traffic.md")
    if not os.path.exists(note):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for line in open(note):
        m = re.match(r"traffic: kernel=(\S+) recipe=(\S+) dtype=(\S+) bytes_per_launch=([0-9.eE+]+) "
                     r"source_sha256=([0-9a-f]+)", line)
        if m and m.group(1) == kernel and m.group(2) == recipe and m.group(3) == dtype_name and m.group(5) == sha:
            return float(m.group(4))
    return None


def main():
    args = parse()
    if args.mode == "wave":
        return run_wave_only(args)
    if args.mode == "copy":
        return run_copy_only(args)
    if args.mode == "stream":
        return run_stream(args)
    if args.mode == "serve":
        return run_serve(args)
    if args.mode == "precision":
        return run_precision(args)
    if args.mode == "paper2d":
        return run_paper2d(args)
    if args.gpus != 1:
        print(json.dumps({"error": "ffpat runs on one GPU; --gpus must be 1 "
                                   "(z-slab sharding across GPUs is designed, not built)"}))
        sys.exit(2)
    import torch
    import paper_1901_06503_amd as ff
    import synth

    dtype = torch.float32 if args.dtype == "float32" else torch.float64
    log(f"inputs {args.recipe} {args.dtype}")
    case, plan, G = make_inputs(args, torch, ff, synth, dtype)
    N, nang = case.n, len(case.angles)
    log(f"N={N} angles={nang} nt={plan.nt} dt={plan.dt:.6g}")
    t, t_power, out = time_fb(torch, plan, G, case.lam, args.steps, args.warmup, args.reg)
    ms = 1e3 * t / args.steps
    log(f"FB {args.steps} iterations: {t:.3f}s ({ms:.2f} ms/iter), power iteration {t_power:.3f}s")

    roof = stencil_roofline(torch, ff, plan, torch.from_numpy(case.c).to("cuda", dtype), case.dx, case.T,
                            case.angles, dtype)
    t_launch = roof["t_launch"]
    achieved = roof["alg_bytes"] / t_launch / 1e9
    achieved_c = roof["compulsory_bytes"] / t_launch / 1e9
    gpt = N ** 3 * plan.nt / roof["t_wave"] / 1e9
    log(f"{roof['kernel']} {t_launch * 1e6:.1f} us/launch, {achieved:.0f} GB/s algorithmic, "
        f"{achieved_c:.0f} GB/s compulsory; W_T {roof['t_wave'] * 1e3:.2f} ms, {gpt:.1f} Gpt-updates/s")
    ceiling = (stream_ceiling(torch, roof["compulsory_bytes"], achieved_c)
               if roof["kernel"] != "wave_step_blocked" else None)
    log(f"streaming ceiling of the same streams: {ceiling}")

    fp64 = None
    G_keep = G.cpu() if args.cpu_baseline else None
    if args.fp64_compare and dtype == torch.float32:
        plan.close()
        del G
        torch.cuda.empty_cache()
        case64, plan64, G64 = make_inputs(args, torch, ff, synth, torch.float64)
        k64 = max(10, args.steps // 2)
        t64, _, _ = time_fb(torch, plan64, G64, case.lam, k64, 2)
        fp64 = {"fb_iter_per_s": k64 / t64, "ms_per_iter": 1e3 * t64 / k64, "steps": k64,
                "wave_gpt_updates_per_s": N ** 3 * plan64.nt / time_wave(torch, plan64) / 1e9,
                "steps_per_pass": plan64.steps_per_pass}
        plan64.close()
        log(f"FP64: {fp64}")

    cpu = None
    if args.cpu_baseline:
        log("cpu baseline (oracle, one FB iteration)")
        cpu = cpu_baseline(case, G_keep, out.step)
        log(f"cpu baseline {cpu}")
    traffic = stored_traffic(roof["kernel"], args.recipe, args.dtype)

    op384 = None
    if args.operator_384 and args.recipe == "c256":
        log("forward operator at 384^3 (FP32, FP64)")
        op384 = operator_384(torch, ff, synth, args.seed + 1000)

    serve = None
    if args.serve_jobs > 0:
        log(f"serving leg: {args.serve_jobs} jobs at 4 jobs/s")
        try:
            sv = serve_summary(args.serve_jobs, 4.0, 50, args.slots, args.concurrency, args.policy,
                               args.fill_voxels, 1, args.seed, args.aging, args.low_concurrency,
                               args.backlog, args.join_voxels)
            cb, se = sv["continuous_batching"], sv["serial"]
            serve = {"trace": f"{args.serve_jobs} jobs, Poisson 4 jobs/s, grids 64^3..256^3, 50 FB iterations each, "
                              f"FP32, policy {args.policy}",
                     "throughput_gain": sv["throughput_gain"],
                     "latency_p50_s": cb["latency_p50_s"], "latency_p99_s": cb["latency_p99_s"],
                     "jobs_per_s": cb["jobs_per_s"], "serial_latency_p50_s": se["latency_p50_s"],
                     "serial_latency_p99_s": se["latency_p99_s"], "serial_jobs_per_s": se["jobs_per_s"],
                     "gpu_busy_mean_pct": cb.get("gpu_busy_mean_pct"),
                     "serial_gpu_busy_mean_pct": se.get("gpu_busy_mean_pct")}
        except Exception as e:          # the serving leg never costs the benchmark line
            serve = {"error": f"{type(e).__name__}: {e}"}
        log(f"serving {serve}")
    serve_sat = None
    if args.serve_jobs > 0 and args.serve_saturated_jobs > 0:
        log(f"saturated serving leg: {args.serve_saturated_jobs} jobs at 8 jobs/s")
        try:
            sv = serve_summary(args.serve_saturated_jobs, 8.0, 50, args.slots, args.concurrency, args.policy,
                               args.fill_voxels, 1, args.seed + 1, args.aging, args.low_concurrency,
                               args.backlog, args.join_voxels)
            cb, se = sv["continuous_batching"], sv["serial"]
            serve_sat = {"trace": f"{args.serve_saturated_jobs} jobs, Poisson 8 jobs/s, grids 64^3..256^3, "
                                  f"50 FB iterations each, FP32, policy {args.policy}",
                         "throughput_gain": sv["throughput_gain"], "jobs_per_s": cb["jobs_per_s"],
                         "serial_jobs_per_s": se["jobs_per_s"], "latency_p50_s": cb["latency_p50_s"],
                         "latency_p99_s": cb["latency_p99_s"], "serial_latency_p50_s": se["latency_p50_s"],
                         "serial_latency_p99_s": se["latency_p99_s"],
                         "gpu_busy_mean_pct": cb.get("gpu_busy_mean_pct"),
                         "serial_gpu_busy_mean_pct": se.get("gpu_busy_mean_pct")}
        except Exception as e:          # never costs the benchmark line
            serve_sat = {"error": f"{type(e).__name__}: {e}"}
        log(f"saturated serving {serve_sat}")

    line = {
        "metric": METRIC,
        "value": args.steps / t,
        "unit": "FB iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic (seeded phantom: balls + tubes, smoothed; c: Gaussian bumps)",
        "config": {"workload": f"{N}^3 grid, {nang} angles, T={case.T}, Algorithm 8 with "
                               + (f"positivity + lambda={case.lam} l2 prox, " if args.reg == "l2" else
                                  f"lambda={case.lam} gradient regulariser (CG prox), ")
                               + ("FP32 fields + FP64 reductions" if dtype == torch.float32 else "all-FP64"),
                   "grid": N, "angles": nang, "nt": plan.nt, "power_steps": 20,
                   "stencil": "naive" if args.naive_stencil else roof["kernel"]},
        "wave_gpt_updates_per_s": gpt,
        "power_iteration_s": t_power,
        "fp64": fp64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": roof["kernel"], "bytes_per_launch": roof["alg_bytes"],
                     "byte_unit": f"algorithmic: 16 B per point update (FP32; read p(k), p(k-1), k', write "
                                  f"p(k+1)) x {roof['updates_per_launch']} update(s) per voxel per launch",
                     "avg_launch_us": t_launch * 1e6,
                     "compulsory": {"bytes_per_launch": roof["compulsory_bytes"], "achieved": achieved_c,
                                    "frac": achieved_c / HBM_PEAK_GBS,
                                    "byte_unit": "words a launch must move per voxel (5 for two or three "
                                                 "steps: read p(k-1), p(k), k', write the last two levels)"},
                     "stream_ceiling": ceiling,
                     "target": "the >= 0.60 HBM target applies to the operator HBM fraction of A = X W_T at "
                               "384^3 (operator_384.*.operator_hbm_frac, beyond the 256 MB MALL)"},
        "operator_384": op384,
        "cpu_baseline": cpu,
        "serving": serve,
        "serving_saturated": serve_sat,
        "objective_last": float(out.objective[-1]) if len(out.objective) else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

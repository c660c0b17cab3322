"""Writes the golden fixtures of the full-size parity tests.  Calls only the
oracle and the seeded input generators (no HIP code).

  python tests/golden/make_golden.py c128   # 128^3 reconstruction, 100 iterations
  python tests/golden/make_golden.py c256   # 256^3 forward / adjoint / gradient samples
  python tests/golden/make_golden.py c384crop  # 64^3 window of the 384^3 workload, 200 iterations

Each fixture is a small JSON text file: the recipe, seeds, sample indices and
the oracle's values there.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402

N_SAMPLES = 4096


def sample_indices(shape, seed, count=N_SAMPLES):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=count, replace=False))


def as_f32_values(case):
    """c and h_true rounded to FP32: the values an FP32 plan holds, exactly
    representable in FP64, so FP32 and FP64 plans see the same c_max and n_t."""
    case.c = case.c.astype(np.float32).astype(np.float64)
    case.h_true = case.h_true.astype(np.float32).astype(np.float64)
    return case


def geometry(case):
    n = case.n
    return oracle.Geometry(nx=n, ny=n, nz=n, dx=case.dx, T=case.T, angles=case.angles)


def simulate(case, g):
    """G = A h_true + eta * mean(A h_true) * n (Sec. 4.2 noise convention)."""
    clean = oracle.forward(g, case.c, case.h_true)
    G = clean + case.noise_level * float(np.mean(clean)) * case.noise
    return G.astype(np.float32).astype(np.float64)


def make_c128(seed=2001):
    case = as_f32_values(synth.make_case("c128", seed))
    g = geometry(case)
    t0 = time.time()
    G = simulate(case, g)
    h, obj, step = oracle.fb(g, case.c, G, case.lam, step=0.0, n_iter=case.n_iter, n_power=case.n_power,
                             flags=oracle.POSITIVITY | oracle.PRECOND)
    idx = sample_indices(g.vol_shape, seed + 1)
    err = float(np.linalg.norm(h - case.h_true) / np.linalg.norm(case.h_true))
    return {"recipe": "c128", "seed": seed, "sample_seed": seed + 1, "n_iter": case.n_iter, "n_power": case.n_power,
            "lam": case.lam, "step": step, "objective": obj.tolist(), "h_norm": float(np.linalg.norm(h)),
            "sample_index": idx.tolist(), "h_sample": h.ravel()[idx].tolist(),
            "relative_error_vs_phantom": err, "oracle_seconds": time.time() - t0}


def make_c256(seed=3001):
    case = as_f32_values(synth.make_case("c256", seed))
    g = geometry(case)
    t0 = time.time()
    fwd = oracle.forward(g, case.c, case.h_true)
    data_rand = synth.random_field(g.data_shape, seed + 10).astype(np.float32).astype(np.float64)
    adj = oracle.adjoint(g, case.c, data_rand)
    # gradient of 1/2 ||A h - d||^2 at h = h_true with d = data_rand (both synthetic inputs)
    grad = oracle.adjoint(g, case.c, fwd - data_rand)
    n = case.n
    c0 = n // 2 - 8
    crop = grad[c0:c0 + 16, c0:c0 + 16, c0:c0 + 16]
    fi = sample_indices(g.data_shape, seed + 2)
    ai = sample_indices(g.vol_shape, seed + 3)
    return {"recipe": "c256", "seed": seed, "data_seed": seed + 10, "crop_origin": c0, "crop_size": 16,
            "forward_index": fi.tolist(), "forward_sample": fwd.ravel()[fi].tolist(),
            "forward_norm": float(np.linalg.norm(fwd)),
            "adjoint_index": ai.tolist(), "adjoint_sample": adj.ravel()[ai].tolist(),
            "adjoint_norm": float(np.linalg.norm(adj)),
            "gradient_crop": crop.ravel().tolist(), "gradient_norm": float(np.linalg.norm(grad)),
            "oracle_seconds": time.time() - t0}


def make_c384crop(seed=4001):
    """The central 64^3 window of the 384^3 workload as a standalone problem (same
    dx = 3/383, T = 0.6, 360 angles, 10 bumps clamped to [0.75, 1.25]); 200 FB
    iterations after a 20-step power iteration."""
    case = as_f32_values(synth.make_case("c384", seed, n=64, dx=synth.grid_spacing(384)))
    g = geometry(case)
    t0 = time.time()
    G = simulate(case, g)
    h, obj, step = oracle.fb(g, case.c, G, case.lam, step=0.0, n_iter=case.n_iter, n_power=case.n_power,
                             flags=oracle.POSITIVITY | oracle.PRECOND)
    err = float(np.linalg.norm(h - case.h_true) / np.linalg.norm(case.h_true))
    idx = sample_indices(g.vol_shape, seed + 1, count=8192)
    return {"recipe": "c384", "window": 64, "seed": seed, "sample_seed": seed + 1, "n_iter": case.n_iter,
            "n_power": case.n_power, "lam": case.lam, "step": step, "objective": obj.tolist(),
            "h_norm": float(np.linalg.norm(h)), "sample_index": idx.tolist(), "h_sample": h.ravel()[idx].tolist(),
            "relative_error_vs_phantom": err, "oracle_seconds": time.time() - t0}


if __name__ == "__main__":
    which = sys.argv[1]
    out = {"c128": make_c128, "c256": make_c256, "c384crop": make_c384crop}[which]()
    path = os.path.join(HERE, f"{which}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({out['oracle_seconds']:.0f} s of oracle time)")

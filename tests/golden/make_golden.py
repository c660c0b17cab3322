"""Writes the golden fixtures of the full-size parity tests.  Calls only the
oracle and the seeded input generators (no HIP code).

  python tests/golden/make_golden.py c128   # 128^3 reconstruction, 100 iterations
  python tests/golden/make_golden.py c256   # 256^3 forward / adjoint / gradient
  python tests/golden/make_golden.py c384crop  # 64^3 window of the 384^3 workload, 200 iterations

Each fixture is a JSON text file (the recipe, seeds, sample indices and the
oracle's values there, scalars) and an .npz file beside it (arrays, loaded with
numpy's default allow_pickle=False): norms of every row and column of the
outputs, complete planes next to the z-chunk boundaries of the two-step stencil
kernel at these sizes, the 32^3 gradient crop and the complete 64^3 window iterate.
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

# z-planes stored whole at 256^3: the grid's first and last plane and both sides of
# the 32- and 64-plane chunk boundaries (FP32 groups march 32 planes, FP64 64)
C256_PLANES = (0, 31, 32, 63, 64, 255)
# 128^3: groups of both precisions march 8 planes; one boundary in the middle
C128_PLANES = (63, 64)


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


def line_norms(a):
    """L2 norms of a 3D array along its last axis and along its middle axis: for a
    volume [z][y][x] the norms of every x-row and every y-column of each plane, for
    data [angle][z][s] those of every detector row and of every (z, s) over angles
    (axis 0) instead of the middle axis."""
    return np.sqrt(np.sum(a * a, axis=-1)), np.sqrt(np.sum(a * a, axis=-2))


def data_norms(a):
    return np.sqrt(np.sum(a * a, axis=-1)), np.sqrt(np.sum(a * a, axis=0))


def make_c128(seed=2001):
    case = as_f32_values(synth.make_case("c128", seed))
    g = geometry(case)
    t0 = time.time()
    G = simulate(case, g)
    h, obj, step = oracle.fb(g, case.c, G, case.lam, step=0.0, n_iter=case.n_iter, n_power=case.n_power,
                             flags=oracle.POSITIVITY | oracle.PRECOND)
    idx = sample_indices(g.vol_shape, seed + 1)
    err = float(np.linalg.norm(h - case.h_true) / np.linalg.norm(case.h_true))
    rows, cols = line_norms(h)
    arrays = {"h_row_norms": rows, "h_col_norms": cols, "h_planes": h[list(C128_PLANES)]}
    meta = {"recipe": "c128", "seed": seed, "sample_seed": seed + 1, "n_iter": case.n_iter,
            "n_power": case.n_power, "lam": case.lam, "step": step, "objective": obj.tolist(),
            "h_norm": float(np.linalg.norm(h)), "sample_index": idx.tolist(), "h_sample": h.ravel()[idx].tolist(),
            "planes": list(C128_PLANES), "relative_error_vs_phantom": err, "oracle_seconds": time.time() - t0}
    return meta, arrays


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
    m = 32
    c0 = n // 2 - m // 2
    crop = grad[c0:c0 + m, c0:c0 + m, c0:c0 + m]
    fi = sample_indices(g.data_shape, seed + 2)
    ai = sample_indices(g.vol_shape, seed + 3)
    planes = list(C256_PLANES)
    f_rows, f_cols = data_norms(fwd)
    a_rows, a_cols = line_norms(adj)
    arrays = {
        # complete planes, rounded to FP32 for size (relative rounding <= 2^-24)
        "forward_planes": np.ascontiguousarray(fwd[:, planes, :].transpose(1, 0, 2)).astype(np.float32),
        "adjoint_planes": adj[planes].astype(np.float32),
        "forward_row_norms": f_rows, "forward_col_norms": f_cols,
        "adjoint_row_norms": a_rows, "adjoint_col_norms": a_cols,
        "gradient_crop": crop,
    }
    meta = {"recipe": "c256", "seed": seed, "data_seed": seed + 10, "crop_origin": c0, "crop_size": m,
            "planes": planes,
            "forward_index": fi.tolist(), "forward_sample": fwd.ravel()[fi].tolist(),
            "forward_norm": float(np.linalg.norm(fwd)),
            "adjoint_index": ai.tolist(), "adjoint_sample": adj.ravel()[ai].tolist(),
            "adjoint_norm": float(np.linalg.norm(adj)),
            "gradient_norm": float(np.linalg.norm(grad)),
            "oracle_seconds": time.time() - t0}
    return meta, arrays


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
    meta = {"recipe": "c384", "window": 64, "seed": seed, "sample_seed": seed + 1, "n_iter": case.n_iter,
            "n_power": case.n_power, "lam": case.lam, "step": step, "objective": obj.tolist(),
            "h_norm": float(np.linalg.norm(h)), "sample_index": idx.tolist(), "h_sample": h.ravel()[idx].tolist(),
            "relative_error_vs_phantom": err, "oracle_seconds": time.time() - t0}
    return meta, {"h": h}


if __name__ == "__main__":
    which = sys.argv[1]
    meta, arrays = {"c128": make_c128, "c256": make_c256, "c384crop": make_c384crop}[which]()
    path = os.path.join(HERE, f"{which}_oracle.json")
    with open(path, "w") as f:
        json.dump(meta, f)
    np.savez_compressed(os.path.join(HERE, f"{which}_oracle.npz"), **arrays)
    print(f"wrote {path} and its .npz ({meta['oracle_seconds']:.0f} s of oracle time)")

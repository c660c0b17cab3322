"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This module produces inputs only (phantoms h, sound speeds c, angle sets,
standard-normal noise fields).  It contains none of the reconstruction
method's arithmetic: no wave solve, projection, filter or iteration.

Stand-ins for the paper's inputs: the paper's own phantom and trapping sound
speed (Sec. 4.2, Fig. 1) exist only as figures, so seeded synthetic phantoms
of the same kind (smoothed balls and thin vessel-like tubes) and smooth
sound-speed bumps are used instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DOMAIN_HALF_WIDTH = 1.5  # the domain is [-1.5, 1.5]^3


def grid_spacing(n: int, half_width: float = DOMAIN_HALF_WIDTH) -> float:
    """Node-centred grid covering [-L, L] with n nodes, endpoints included."""
    return 2.0 * half_width / (n - 1)


def axis(n: int, dx: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * dx


def uniform_angles(n_angles: int) -> np.ndarray:
    """phi_a = a pi / n_angles, a = 0..n_angles-1 (uniform in [0, pi))."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


def _uniform_in_ball(rng, radius, count):
    pts = []
    while len(pts) < count:
        p = rng.uniform(-radius, radius, size=3)
        if p @ p <= radius * radius:
            pts.append(p)
    return np.array(pts).reshape(count, 3)


def _coords(shape, dx):
    nz, ny, nx = shape
    z = axis(nz, dx)[:, None, None]
    y = axis(ny, dx)[None, :, None]
    x = axis(nx, dx)[None, None, :]
    return z, y, x


def gaussian_smooth(vol: np.ndarray, sigma_vox: float = 1.0, axes=(0, 1, 2)) -> np.ndarray:
    """Separable Gaussian blur over `axes` (sigma in voxels, truncated at 4 sigma, zero padded,
    unit-sum kernel)."""
    if sigma_vox <= 0:
        return vol.copy()
    r = int(math.ceil(4 * sigma_vox))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sigma_vox) ** 2)
    k /= k.sum()
    out = vol.astype(np.float64, copy=True)
    for ax in axes:
        pad = [(0, 0)] * 3
        pad[ax] = (r, r)
        padded = np.pad(out, pad)
        acc = np.zeros_like(out)
        n = out.shape[ax]
        for i, w in enumerate(k):
            sl = [slice(None)] * 3
            sl[ax] = slice(i, i + n)
            acc += w * padded[tuple(sl)]
        out = acc
    return out


def balls(shape, dx, rng, n_balls, centre_radius=0.8, radii=(0.1, 0.3), values=(0.5, 1.0)):
    """Union (by max) of uniform balls with seeded centres, radii and values."""
    z, y, x = _coords(shape, dx)
    vol = np.zeros(shape)
    centres = _uniform_in_ball(rng, centre_radius, n_balls)
    rad = rng.uniform(*radii, size=n_balls)
    val = rng.uniform(*values, size=n_balls)
    for (cx, cy, cz), r, v in zip(centres, rad, val):
        inside = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
        vol = np.maximum(vol, np.where(inside, v, 0.0))
    return vol


def tubes(shape, dx, rng, n_tubes, centre_radius=0.8, n_vertices=(3, 6), seg_len=(0.1, 0.3),
          radius_vox=(1.0, 2.0), values=(0.5, 1.0)):
    """Thin vessel-like tubes: random polylines rasterised by distance to segment."""
    nz, ny, nx = shape
    vol = np.zeros(shape)
    ax_ = [axis(nz, dx), axis(ny, dx), axis(nx, dx)]
    for _ in range(n_tubes):
        nv = int(rng.integers(n_vertices[0], n_vertices[1] + 1))
        p = _uniform_in_ball(rng, centre_radius, 1)[0]
        verts = [p]
        for _ in range(nv - 1):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            verts.append(verts[-1] + rng.uniform(*seg_len) * d)
        rad = rng.uniform(*radius_vox) * dx
        val = rng.uniform(*values)
        for a, b in zip(verts[:-1], verts[1:]):
            lo = np.minimum(a, b) - rad
            hi = np.maximum(a, b) + rad
            # index box (x, y, z order in the vertices; arrays are [z][y][x])
            idx = []
            for dim, arr in zip((2, 1, 0), ax_):
                i0 = int(np.searchsorted(arr, lo[dim], side="left"))
                i1 = int(np.searchsorted(arr, hi[dim], side="right"))
                idx.append((max(i0, 0), min(i1, len(arr))))
            (z0, z1), (y0, y1), (x0, x1) = idx
            if z0 >= z1 or y0 >= y1 or x0 >= x1:
                continue
            Z = ax_[0][z0:z1, None, None]
            Y = ax_[1][None, y0:y1, None]
            X = ax_[2][None, None, x0:x1]
            ab = b - a
            L2 = float(ab @ ab)
            t = ((X - a[0]) * ab[0] + (Y - a[1]) * ab[1] + (Z - a[2]) * ab[2]) / max(L2, 1e-30)
            t = np.clip(t, 0.0, 1.0)
            d2 = (X - a[0] - t * ab[0]) ** 2 + (Y - a[1] - t * ab[1]) ** 2 + (Z - a[2] - t * ab[2]) ** 2
            blk = vol[z0:z1, y0:y1, x0:x1]
            vol[z0:z1, y0:y1, x0:x1] = np.maximum(blk, np.where(d2 <= rad * rad, val, 0.0))
    return vol


def sound_speed(shape, dx, rng, n_bumps, amplitude, clamp, sigma=0.4, centre_radius=1.0):
    """c = 1 + amplitude * sum_i a_i exp(-|r - r_i|^2 / (2 sigma^2)), clamped."""
    z, y, x = _coords(shape, dx)
    c = np.ones(shape)
    centres = _uniform_in_ball(rng, centre_radius, n_bumps)
    amps = rng.uniform(-1.0, 1.0, size=n_bumps)
    for (cx, cy, cz), a in zip(centres, amps):
        c += amplitude * a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * sigma * sigma))
    return np.clip(c, clamp[0], clamp[1])


@dataclass
class Case:
    """One synthetic reconstruction case (inputs only)."""
    n: int
    dx: float
    T: float
    angles: np.ndarray
    h_true: np.ndarray
    c: np.ndarray
    noise: np.ndarray       # standard-normal field of the data shape
    noise_level: float      # eta: sigma = eta * mean(A h_true)
    lam: float
    n_iter: int
    n_power: int

    @property
    def data_shape(self):
        return (len(self.angles), self.n, self.n)


# Workload recipes (grid edge, angles, phantom, sound speed, T, noise, FB settings)
RECIPES = {
    "c48_f64": dict(n=48, n_angles=48, balls=3, tubes=0, bumps=2, amp=0.1, clamp=(0.85, 1.15),
                    T=0.5, eta=0.01, lam=1e-3, n_iter=5, n_power=20),
    "c128": dict(n=128, n_angles=128, balls=20, tubes=200, bumps=5, amp=0.2, clamp=(0.8, 1.2),
                 T=0.5, eta=0.02, lam=1e-3, n_iter=100, n_power=20),
    "c256": dict(n=256, n_angles=256, balls=20, tubes=200, bumps=5, amp=0.2, clamp=(0.8, 1.2),
                 T=0.5, eta=0.02, lam=1e-3, n_iter=100, n_power=20),
    "c384": dict(n=384, n_angles=360, balls=20, tubes=200, bumps=10, amp=0.2, clamp=(0.75, 1.25),
                 T=0.6, eta=0.02, lam=1e-3, n_iter=200, n_power=20),
}


def make_case(recipe: str, seed: int, n: int | None = None, n_angles: int | None = None,
              dx: float | None = None) -> Case:
    """Builds a seeded case from a recipe; n / n_angles override the grid and angle
    count, dx the spacing (with n < the recipe's grid and the recipe's dx this is
    the central n^3 window of the recipe's domain: a standalone sub-problem)."""
    r = dict(RECIPES[recipe])
    if n is not None:
        r["n"] = n
    if n_angles is not None:
        r["n_angles"] = n_angles
    N = r["n"]
    dx = grid_spacing(N) if dx is None else dx
    rng = np.random.default_rng(seed)
    shape = (N, N, N)
    h = balls(shape, dx, rng, r["balls"])
    if r["tubes"]:
        h = np.maximum(h, tubes(shape, dx, rng, r["tubes"]))
    h = gaussian_smooth(h, 1.0)
    c = sound_speed(shape, dx, rng, r["bumps"], r["amp"], r["clamp"])
    noise = rng.standard_normal((r["n_angles"], N, N))
    return Case(n=N, dx=dx, T=r["T"], angles=uniform_angles(r["n_angles"]), h_true=h, c=c,
                noise=noise, noise_level=r["eta"], lam=r["lam"], n_iter=r["n_iter"], n_power=r["n_power"])


def random_field(shape, seed, dtype=np.float64):
    """i.i.d. standard-normal field (for dot tests and parity cases)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def gaussian_blob(shape, dx, centre, sigma, amplitude=1.0):
    """A * exp(-|r - r0|^2 / (2 sigma^2)) sampled on the node-centred grid."""
    z, y, x = _coords(shape, dx)
    cx, cy, cz = centre
    return amplitude * np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * sigma * sigma))


def torch_case(n, n_angles, seed, device="cuda", dtype=None, n_balls=20, n_bumps=5, amp=0.2, clamp=(0.8, 1.2)):
    """Device-side generator for large traces (serving): the recipe's balls
    (smoothed, sigma = 1 voxel) and sound-speed bumps, drawn from a seeded
    numpy generator and rasterised with torch on the device.  Returns
    (dx, angles, c, h) with c, h device tensors [n][n][n]."""
    import torch
    dtype = dtype or torch.float32
    rng = np.random.default_rng(seed)
    dx = grid_spacing(n)
    ax = torch.as_tensor(axis(n, dx), device=device, dtype=torch.float32)
    z, y, x = ax[:, None, None], ax[None, :, None], ax[None, None, :]
    h = torch.zeros((n, n, n), device=device, dtype=torch.float32)
    centres = _uniform_in_ball(rng, 0.8, n_balls)
    rad = rng.uniform(0.1, 0.3, size=n_balls)
    val = rng.uniform(0.5, 1.0, size=n_balls)
    for (cx, cy, cz), r, v in zip(centres, rad, val):
        inside = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
        h = torch.maximum(h, inside.to(torch.float32) * float(v))
    t = torch.arange(-4, 5, device=device, dtype=torch.float32)
    k = torch.exp(-0.5 * t * t)
    k = k / k.sum()
    for dim in range(3):
        pad = [0, 0, 0, 0, 0, 0]
        pad[2 * (2 - dim)] = pad[2 * (2 - dim) + 1] = 4
        hp = torch.nn.functional.pad(h, pad)
        acc = torch.zeros_like(h)
        for i in range(9):
            acc += k[i] * hp.narrow(dim, i, n)
        h = acc
    c = torch.ones((n, n, n), device=device, dtype=torch.float32)
    bc = _uniform_in_ball(rng, 1.0, n_bumps)
    ba = rng.uniform(-1.0, 1.0, size=n_bumps)
    for (cx, cy, cz), a in zip(bc, ba):
        c += amp * float(a) * torch.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * 0.16))
    c = torch.clamp(c, clamp[0], clamp[1])
    return dx, uniform_angles(n_angles), c.to(dtype), h.to(dtype)


def paper2d_case(seed, n=601, half_width=3.0, n_angles=1000, n_disks=12, c_bumps=4, c_amp=0.3):
    """Inputs in the geometry of the paper's 2D experiment (Sec. 4.1): wave grid n x n
    on [-3, 3]^2, source supported in [-1, 1]^2, 1000 angles in [0, pi).  The paper's
    phantom and trapping speed are not available: smoothed disks inside the unit disk
    and smooth Gaussian sound-speed bumps stand in for them.  Arrays are [1][n][n]."""
    rng = np.random.default_rng(seed)
    dx = 2.0 * half_width / (n - 1)
    ax = axis(n, dx)
    y, x = ax[:, None], ax[None, :]
    h = np.zeros((n, n))
    for _ in range(n_disks):
        while True:
            cx, cy = rng.uniform(-0.75, 0.75, size=2)
            if cx * cx + cy * cy <= 0.75 ** 2:
                break
        r = rng.uniform(0.05, 0.2)
        v = rng.uniform(0.5, 1.0)
        h = np.maximum(h, np.where((x - cx) ** 2 + (y - cy) ** 2 <= r * r, v, 0.0))
    h = gaussian_smooth(h[None], 1.0, axes=(1, 2))[0]
    c = np.ones((n, n))
    for _ in range(c_bumps):
        cx, cy = rng.uniform(-1.0, 1.0, size=2)
        c += c_amp * rng.uniform(-1.0, 1.0) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.3 ** 2))
    c = np.clip(c, 0.7, 1.3)
    support = ((np.abs(x) <= 1.0) & (np.abs(y) <= 1.0)).astype(np.uint8)
    noise = rng.standard_normal((n_angles, 1, n))
    return dict(dx=dx, T=2.0, angles=uniform_angles(n_angles), h=h[None], c=c[None], support=support[None],
                noise=noise, stripe=1.0)

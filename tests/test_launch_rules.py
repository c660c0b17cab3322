"""Host logic: the launch-shape rules of the leapfrog stencil kernels.

The rules (csrc/launch_rules.h) are plain arithmetic on the grid, the element size,
the device's compute units and the work-groups a unit holds at once; the library
feeds them the runtime's figures.  A small C++ driver compiled here with g++ runs
the same header on the host.  Expected shapes are for MI355X (256 compute units;
two 64 x 16 FP32 groups per unit, one 128 x 16 FP32 group, one FP64 group): the
picks that were measured fastest among the candidates swept on that device, and the
ones the GPU tests assert through ffpat_plan_stencil_shape.  The driver also reports
whether FP32 runs over pairs of x-adjacent points per lane (the 128 x 16 tile with even
nx; the tile is then given in points and the group count is the pairs kernel's).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1901_06503_amd", "csrc")


@pytest.fixture(scope="module")
def cli(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("rules") / "launch_rules_cli")
    extra = os.environ.get("FFPAT_TEST_HOST_CFLAGS", "").split()   # the sanitizer run adds -fsanitize=...
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + CSRC] + extra +
                   [os.path.join(HERE, "launch_rules_cli.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, *args):
    out = subprocess.run([exe] + [str(a) for a in args], check=True, capture_output=True, text=True).stdout
    return tuple(int(v) for v in out.split())


def pair(exe, nz, ny, nx, f64):
    return _run(exe, "pair", nx, ny, nz, 8 if f64 else 4, 256, 1 if f64 else 2, 1)


# (nz, ny, nx): (tile width in points, planes per group, pairs of x-adjacent points
# per lane) on 256 compute units
PAIR_FP32 = {
    (128, 128, 128): (64, 8, 0), (160, 160, 160): (64, 10, 0), (192, 192, 192): (64, 14, 0),
    (224, 224, 224): (128, 25, 1), (256, 256, 256): (128, 32, 1), (288, 288, 288): (128, 32, 1),
    (320, 320, 320): (64, 32, 0), (384, 384, 384): (128, 55, 1), (448, 448, 448): (128, 50, 1),
    (512, 512, 512): (128, 64, 1), (640, 640, 640): (128, 64, 1),
    (96, 250, 250): (128, 12, 1), (97, 380, 383): (128, 33, 0),   # odd nx: one point per lane
}
PAIR_FP64 = {
    (128, 128, 128): 8, (160, 160, 160): 20, (192, 192, 192): 28, (224, 224, 224): 56,
    (256, 256, 256): 64, (320, 320, 320): 64, (384, 384, 384): 55, (448, 448, 448): 50,
    (512, 512, 512): 64, (97, 380, 383): 20,
}


@pytest.mark.parametrize("shape", sorted(PAIR_FP32))
def test_two_step_fp32_tile_and_chunk(cli, shape):
    bx, by, zc, groups, pairs = pair(cli, *shape, f64=False)
    assert (bx, zc, pairs) == PAIR_FP32[shape] and by == 16


@pytest.mark.parametrize("shape", sorted(PAIR_FP64))
def test_two_step_fp64_chunk(cli, shape):
    bx, by, zc, groups, pairs = pair(cli, *shape, f64=True)
    assert (bx, by, zc, pairs) == (64, 16, PAIR_FP64[shape], 0)


@pytest.mark.parametrize("n", [128, 160, 192, 224, 256])
def test_two_step_fills_one_round_where_it_can(cli, n):
    """Below the point where the longest chunk is needed, the groups fit in one round
    of resident groups and the chunk is the shortest that does (8 planes at least)."""
    for f64 in (False, True):
        bx, by, zc, groups, _ = pair(cli, n, n, n, f64)
        resident = 256 * (1 if (f64 or bx == 128) else 2)
        assert groups <= resident
        if zc > 8:
            xy = -(-n // bx) * -(-n // by)
            assert xy * -(-n // (zc - 1)) > resident


def test_two_step_handles_thin_grids(cli):
    """Fewer planes than the minimum chunk: one chunk of all planes."""
    for nz in (1, 3, 7):
        bx, by, zc, groups, _ = pair(cli, nz, 200, 300, f64=False)
        assert zc == nz


# (nz, ny, nx, esz): (tile height, planes per group) of the one-step kernel
STEP = {
    (256, 256, 256, 4): (8, 16), (384, 384, 384, 4): (16, 16), (64, 64, 64, 4): (8, 1),
    (112, 112, 112, 4): (8, 2), (64, 64, 64, 8): (8, 1), (256, 256, 256, 8): (16, 8),
    (48, 48, 48, 8): (8, 1), (3, 40, 40, 4): (8, 1),
}


@pytest.mark.parametrize("key", sorted(STEP))
def test_one_step_tile_and_chunk(cli, key):
    nz, ny, nx, esz = key
    tx, ty, zc = _run(cli, "step", nx, ny, nz, esz)
    assert (tx, ty, zc) == (64,) + STEP[key]


def test_three_step_1024_thread_slot_layout(cli):
    """The slot layout of the 1024-thread three-step kernel (wide3_interior, wide3_ring,
    wide3_role, wide3_bases): the 1024 interior points are the tile; the ring points of
    each role are exactly the ring of that role (296 around stage 2's region, 312 around
    stage 1's, 328 around the p(k) plane's inner part), so every point of the p(k) plane
    has one kind of slot; every LDS access the kernel makes from those bases (p(k) planes
    with both parities, the five slots of the q and r rings, the stencil's x and y
    neighbours) stays inside its array with an immediate offset below 64 KiB and reads
    or writes the intended element; and the ring stages per plane are spread 4, 4, 4, 3
    over the four SIMDs."""
    out = subprocess.run([cli, "wide3"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.split() == ["ok", "1024", "296", "312", "328"]


# (nz, ny, nx): planes per group of the FP32 three-step pass (128 x 16 point tile) on
# 256 compute units, and whether the grid takes it where the two-step rule keeps the
# 64-point tile or one step per pass
TRIPLE_FP32 = {
    (96, 96, 96): (3, 1), (112, 112, 112): (4, 1), (128, 128, 128): (4, 1), (160, 160, 160): (14, 1),
    (192, 192, 192): (20, 1), (224, 224, 224): (25, 1), (256, 256, 256): (32, 1), (320, 320, 320): (40, 1),
    (384, 384, 384): (55, 1), (512, 512, 512): (64, 1),
    (64, 64, 64): (3, 0),            # too small: one step per pass stays faster
    (130, 130, 130): (10, 0),        # 65 pairs in two 64-pair tiles: half the width idle
    (40, 250, 250): (5, 1),
}


@pytest.mark.parametrize("shape", sorted(TRIPLE_FP32))
def test_three_step_chunk_and_grid_rule(cli, shape):
    nz, ny, nx = shape
    bx, by, zc, groups, ok = _run(cli, "triple", nx, ny, nz, 256)
    assert (bx, by) == (128, 16) and (zc, ok) == TRIPLE_FP32[shape]
    assert groups <= 256 or zc >= 8     # one round of groups where chunks of 3+ planes allow it


def test_three_step_grid_rule_edges(cli):
    assert _run(cli, "triple", 97, 128, 128, 256)[4] == 0    # odd nx: no pairs of points
    assert _run(cli, "triple", 128, 60, 256, 256)[4] == 0    # ny below 64
    assert _run(cli, "triple", 94, 128, 128, 256)[4] == 0    # nx below 96
    assert _run(cli, "triple", 128, 128, 50, 256)[4] == 0    # fewer than 96^3 points

"""Registers, scratch and occupancy of the device kernels, from the compiler's
resource report (CPU only: the device code is compiled for gfx950, nothing runs).

A kernel that spills keeps part of its state in scratch memory and moves it
through the caches on every use.  The three-step FP32 stencil pass (eq. wave1,
three leapfrog steps per launch) once spilled one 8-byte value per lane, which
added 6 MiB of writes per launch at 256^3 and cost 4% of its time.  These tests
fail on any new spill and on an occupancy below what a kernel's launch shape
needs (a 1024-thread work-group is 16 waves: 4 per SIMD)."""
import concurrent.futures as cf
import re
import subprocess

import pytest

pytestmark = pytest.mark.slow

SOURCES = ["kernels_wave.hip", "kernels_xray.hip", "kernels_fb.hip"]

# Kernels allowed to use scratch, with the bytes per lane they may use.
SPILL_ALLOWED = {
    # 128 x 16 FP32 tile for grids with odd nx: its addresses hoisted out of the z
    # loop (one spilled) measured 1-2% faster than recomputing them every plane
    "wave_step2_blocked<float, 3, 4, 1024, 128>": 20,
    # variants reached only through the tuning switches (8-row tiles, 1024-thread
    # FP64 groups); no plan takes them by default
    "wave_step2_blocked<float, 3, 8, 512, 64>": 388,
    "wave_step2_blocked<double, 3, 8, 1024, 64>": 488,
    "wave_step2_blocked<double, 3, 4, 1024, 64>": 140,
    "wave_step2_blocked<double, 3, 8, 512, 64>": 880,
}

# Kernels launched with 1024 threads per work-group: 16 waves on 4 SIMDs.
THREADS_1024 = ("wave_step3_wide<", "project_lds_kernel<", "backproject_lds_kernel<")


def _demangle(names):
    out = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True).stdout
    return dict(zip(names, out.splitlines()))


@pytest.fixture(scope="module")
def report():
    from paper_1901_06503_amd import build
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        parts = list(ex.map(build.device_resource_report, SOURCES))
    merged = {}
    for src, part in zip(SOURCES, parts):
        assert part, f"no resource report for {src}"
        names = _demangle(list(part))
        for mangled, fields in part.items():
            merged[re.sub(r"^void ", "", names[mangled]).split("(")[0]] = fields
    return merged


def _scratch(fields):
    return int(fields["ScratchSize [bytes/lane]"])


def test_report_covers_the_hot_kernels(report):
    for k in ("ffpat::wave_step3_wide<false, false>", "ffpat::wave_step3_wide<true, false>",
              "ffpat::wave_step3_wide<false, true>", "ffpat::project_lds_kernel<float, 8>",
              "ffpat::backproject_lds_kernel<float, 16>", "ffpat::residual_ramp_win_kernel<float>",
              "ffpat::prox_l2_kernel<float>", "ffpat::dst_axis_kernel<float>", "ffpat::dst_axis_kernel<double>"):
        assert k in report, f"{k} missing from the compiler's report"


def test_no_kernel_spills_beyond_the_listed_exceptions(report):
    bad = []
    for name, fields in report.items():
        allowed = SPILL_ALLOWED.get(name.replace("ffpat::", ""), 0)
        if _scratch(fields) > allowed:
            bad.append(f"{name}: {_scratch(fields)} bytes/lane (allowed {allowed})")
    assert not bad, "kernels using scratch:\n" + "\n".join(bad)


def test_the_three_step_pass_uses_no_scratch(report):
    for variant in ("ffpat::wave_step3_wide<false, false>", "ffpat::wave_step3_wide<true, false>",
                    "ffpat::wave_step3_wide<false, true>"):
        f = report[variant]
        assert _scratch(f) == 0 and f.get("VGPRs Spill") == "0", f
        assert int(f["LDS Size [bytes/block]"]) <= 160 * 1024


def test_1024_thread_kernels_reach_four_waves_per_simd(report):
    for name, fields in report.items():
        if name.replace("ffpat::", "").startswith(THREADS_1024):
            assert int(fields["Occupancy [waves/SIMD]"]) >= 4, f"{name}: {fields}"

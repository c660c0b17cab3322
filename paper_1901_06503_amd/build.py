"""Builds libffpat.so (HIP, gfx950) in-tree from csrc/*.hip, and beside it
libffpat_probe.so (the streaming-ceiling kernels the benchmark times).

Usage: python -m paper_1901_06503_amd.build  [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libffpat.so")
ARCH = "gfx950"

SOURCES = ["kernels_wave.hip", "kernels_xray.hip", "kernels_fb.hip", "plan.hip"]
PROBE_LIB = os.path.join(HERE, "libffpat_probe.so")
PROBE_SOURCES = ["stream_probe.hip"]

# Packed FP32 instructions are disabled on purpose: the compiler forms them from
# ordinary float code, and some of their forms have produced silently wrong
# results on this hardware.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libffpat")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc()] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


# roctx ranges of the C ABI calls (rocprofiler-sdk's marker library, beside libamdhip64)
LINK_LIBS = ["-lrocprofiler-sdk-roctx"]


def _link(objs, lib: str, libs=()):
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + list(libs) + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


# Host-side sanitizer build for the CPU tests (no GPU needed): AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (each flag behind -Xarch_host), so
# the argument checks, layouts and launch-shape rules of the C ABI run instrumented.
# The library leaves the sanitizer runtime to the process (preloaded by the test).
SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(jobs: int = 4) -> str:
    """Builds _build/san/libffpat.so with the host code under ASan and UBSan (-O1 -g)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    flags = [f for f in HIP_FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST_FLAGS

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(SAN_DIR, "libffpat.so")
    _link(objs, lib, LINK_LIBS)
    return lib


def device_resource_report(src: str) -> dict:
    """Compiles the device code of csrc/`src` for gfx950 with the library's flags and
    returns the compiler's resource report per kernel: {mangled name: {field: value}},
    fields as the compiler prints them ("VGPRs", "ScratchSize [bytes/lane]",
    "Occupancy [waves/SIMD]", "LDS Size [bytes/block]", ...).  CPU only."""
    import re
    import tempfile
    flags = [f for f in HIP_FLAGS if f != "-fPIC"]
    with tempfile.TemporaryDirectory() as tmp:
        cmd = [hipcc()] + flags + ["--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
                                   "-c", os.path.join(CSRC, src), "-o", os.path.join(tmp, "dev.o")]
        r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    report, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = report.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis=kernel-resource-usage\]", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return report


def build(jobs: int = 4, verbose: bool = False) -> str:
    """Compiles every source (always, also when a library exists) and links
    libffpat.so and libffpat_probe.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, SOURCES + PROBE_SOURCES))
    _link(objs[:len(SOURCES)], LIB, LINK_LIBS)
    _link(objs[len(SOURCES):], PROBE_LIB)
    if verbose:
        print(f"built {LIB}")
        print(f"built {PROBE_LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)

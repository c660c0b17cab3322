"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Three runs, each in a process of its own (one sanitizer runtime per process):

* the oracle built with gcc's sanitizers (oracle.build_sanitized), gcc's runtimes
  preloaded: every CPU test that does not load the HIP library (the oracle's pins,
  the launch-shape rules with their driver built with the same sanitizers, the
  scheduler's policies, the benchmark's host contract);
* the HIP library with its host code under clang's sanitizers
  (build.build_sanitized), clang's ASan runtime preloaded: the C ABI's host checks
  (test_abi.py: validation, layouts, exports, the C99 caller);
* the plain C caller (tests/abi_consumer.c) built with clang's sanitizers and
  linked to that library.

Sanitizer errors are fatal (-fno-sanitize-recover=all, halt_on_error), so a run
passes only if no instrumented access or operation was reported.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtimes():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    libs = [subprocess.run([gcc, f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
            for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in libs):
        pytest.skip("gcc sanitizer runtimes not found")
    return libs


def _clang():
    for cand in ("/opt/rocm/llvm/bin/clang", shutil.which("clang")):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("clang not available")


def _clang_asan_runtime(clang):
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.exists(rt):
        found = glob.glob(os.path.join(os.path.dirname(os.path.dirname(clang)), "lib", "clang", "*", "lib",
                                       "linux", "libclang_rt.asan-x86_64.so"))
        if not found:
            pytest.skip("clang ASan runtime not found")
        rt = found[0]
    return rt


def _pytest(args, env_extra, timeout=900):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow"] + args
    run = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    return run.stdout


def test_oracle_and_host_logic_under_gcc_sanitizers(tmp_path):
    import oracle
    libs = _gcc_runtimes()
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    out = _pytest([os.path.join(TESTS, f) for f in ("test_oracle_wave.py", "test_oracle_xray.py", "test_oracle_fb.py",
                                                     "test_oracle_properties.py", "test_launch_rules.py",
                                                     "test_serving_policy.py", "test_bench_contract.py")],
                  {"LD_PRELOAD": " ".join(libs), "FFPAT_ORACLE_LIB": lib,
                   "FFPAT_TEST_HOST_CFLAGS": "-fsanitize=address,undefined -fno-sanitize-recover=all "
                                             "-fno-omit-frame-pointer"})
    assert " passed" in out and "failed" not in out


@pytest.fixture(scope="module")
def sanitized_library():
    from paper_1901_06503_amd import build
    return build.build_sanitized()


def test_c_abi_host_code_under_clang_sanitizers(sanitized_library):
    rt = _clang_asan_runtime(_clang())
    # the C99 caller of test_abi.py links with gcc and no sanitizer runtime: it is built
    # with clang's sanitizers in the next test instead
    out = _pytest([os.path.join(TESTS, "test_abi.py"), "-k", "not plain_c_caller"],
                  {"LD_PRELOAD": rt, "FFPAT_LIB_PATH": sanitized_library})
    assert " passed" in out and "failed" not in out


def test_plain_c_caller_under_clang_sanitizers(sanitized_library, tmp_path):
    clang = _clang()
    libdir = os.path.dirname(sanitized_library)
    exe = str(tmp_path / "abi_consumer_san")
    subprocess.run([clang, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(TESTS, "abi_consumer.c"), "-L" + libdir, "-lffpat", "-Wl,-rpath," + libdir,
                    "-o", exe], check=True)
    run = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, **SAN_ENV), timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.count("ok ") == 9 and "FAIL" not in run.stdout

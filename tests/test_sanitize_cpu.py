"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (no GPU): the oracle's C
functions (tests/sanitize/oracle_check.c) and the library's host-side table preparation and
argument checking (tests/sanitize/host_check.cpp, which compiles tc_host.cpp with stub kernel
launchers).  Each program must run clean and print "ok"."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", *SAN, "-std=c11", "-fopenmp", "-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "totalconv_oracle.c"), "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="1"))
    assert r.stdout.strip().endswith("ok"), r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")),
                    reason="no g++ or HIP headers")
def test_host_preparation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    _run(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1002_1050_amd", "csrc"),
          "-o", exe, os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
          "-L", os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64"])
    # the HIP runtime's own start-up allocations are not this code's: leaks are checked in
    # the oracle build, memory errors and undefined behaviour here
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1"))
    assert r.stdout.strip().endswith("ok"), r.stdout

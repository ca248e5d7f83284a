"""The planner's worker pool (CPU): repeated, concurrent, nested and
post-fork parallel loops each run every body index exactly once; built
optimized, with AddressSanitizer + UndefinedBehaviorSanitizer and with
ThreadSanitizer (any report fails the run)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1201_5991_amd", "csrc")


BUILDS = {
    "O2": ["-O2"],
    "asan_ubsan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-O1", "-g", "-fsanitize=thread"],
}
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
           "TSAN_OPTIONS": "halt_on_error=1:die_after_fork=0"}


@pytest.mark.parametrize("build", list(BUILDS))
def test_worker_pool(tmp_path, build):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "pool_check")
    cmd = [cxx, *BUILDS[build], "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "pool_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env={**os.environ, **SAN_ENV})
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr

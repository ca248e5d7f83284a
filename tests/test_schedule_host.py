"""Host factorization schedule (CPU): nested-dissection interiors, the tile
structure and the schedule in which groups of one dissection height advance
together.  A small C++ program built from the library's planner runs the task
list of one subdomain in launch order on a random SPD matrix with the
subdomain's element pattern and compares with a dense partial Cholesky of the
interior columns (it also checks that no launch writes a tile twice).  The
program is built twice: optimized, and with AddressSanitizer and
UndefinedBehaviorSanitizer, which abort on any memory or undefined-behaviour
error in the planner."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1201_5991_amd.solver import Problem
from workloads import box_workload
from workloads.gen import uniform_cuts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1201_5991_amd", "csrc")


# Host-only builds of the planner: optimized, and with AddressSanitizer and
# UndefinedBehaviorSanitizer (any report aborts the program).
BUILDS = {
    "O2": ["-O2"],
    "asan_ubsan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
}
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


@pytest.fixture(scope="module", params=list(BUILDS))
def checker(request, tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("sched")
    exe = str(d / "schedule_check")
    cmd = [cxx, *BUILDS[request.param], "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "schedule_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # 3x3x3 subdomains of 9^3 elastic hexahedra: 8^3 interior nodes of the centre
    # subdomain (1536 DOFs) are cut into two parts and a separator
    n = 27
    w = box_workload("sched", "elasticity", (n,) * 3, [uniform_cuts(n, 3)] * 3, groups=(), young=None, seed=0)
    p = Problem(w)
    p.elem_nodes.tofile(d / "elem_nodes.bin")
    p.dirichlet.tofile(d / "dirichlet.bin")
    p.elem_to_sub.tofile(d / "elem_to_sub.bin")
    for i, par in enumerate(p.parents):
        np.asarray(par, dtype=np.int32).tofile(d / f"parent{i}.bin")
    (d / "meta.txt").write_text(f"{p.dim} {p.ndof} {p.n_nodes} {p.n_elems} {p.nodes_per_elem} {p.n_levels} "
                                f"{len(p.parents)} {p.constraints}\n")
    return exe, str(d)


@pytest.mark.parametrize("build", ["asan_ubsan", "tsan"])
def test_layout_reuse_matches_fresh_dissection(tmp_path, build):
    """4x4x4 subdomains of 8^3: the eight interior ones (and the other
    repeated shapes) reuse one dissection; the checker compares every level-1
    layout with a plan that dissects each subdomain afresh, then runs a
    reused subdomain's schedule against the dense Cholesky.  Built with
    ASan + UBSan and with ThreadSanitizer (threads wait for an equal
    structure that another thread is dissecting)."""
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "schedule_check")
    flags = {**BUILDS, "tsan": ["-O1", "-g", "-fsanitize=thread"]}[build]
    cmd = [cxx, *flags, "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "schedule_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    n = 32
    w = box_workload("reuse", "elasticity", (n,) * 3, [uniform_cuts(n, 4)] * 3, groups=(), young=None, seed=0)
    p = Problem(w)
    p.elem_nodes.tofile(tmp_path / "elem_nodes.bin")
    p.dirichlet.tofile(tmp_path / "dirichlet.bin")
    p.elem_to_sub.tofile(tmp_path / "elem_to_sub.bin")
    (tmp_path / "meta.txt").write_text(f"{p.dim} {p.ndof} {p.n_nodes} {p.n_elems} {p.nodes_per_elem} {p.n_levels} "
                                       f"0 {p.constraints}\n")
    sub = 1 + 4 + 16 * 2     # an interior subdomain
    env = {**os.environ, **SAN_ENV, "MLBDDC_VERBOSE": "1", "TSAN_OPTIONS": "halt_on_error=1"}
    r = subprocess.run([exe, str(tmp_path), str(sub), "3"], capture_output=True, text=True, timeout=900, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    reused = [l for l in r.stderr.splitlines() if "layouts reuse" in l]
    assert reused and int(reused[0].split("] ")[1].split()[0]) >= 30, r.stderr[-2000:]


@pytest.mark.parametrize("sub,panel", [(13, 2), (0, 4), (4, 3)])
def test_schedule_reproduces_dense_cholesky(checker, sub, panel):
    exe, d = checker
    r = subprocess.run([exe, d, str(sub), str(panel)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, **SAN_ENV})
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    # the centre subdomain is cut by the dissection (several groups)
    if sub == 13:
        assert int(r.stdout.split(" groups ")[1].split()[0]) >= 3

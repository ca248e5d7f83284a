"""The allocation-free interface-operator entry point (runs on an MI355X).

mlbddc_apply_schur_noalloc computes y = S^ x with its work vectors in the
library's static device scratch array instead of device memory of the
handle.  Through the C ABI, its result is compared with
mlbddc_apply_schur's on two calls in a row, the second on a smaller problem
(the scratch keeps the first call's contents), to relative 1e-10 (FP64,
another summation order), and no device memory is allocated by the call.
"""

import ctypes as C

import numpy as np
import pytest
import torch

from workloads import box_workload
from workloads.gen import uniform_cuts

pytestmark = pytest.mark.gpu


def _cube(n_sub, el, seed):
    n = n_sub * el
    young = 10 ** (2 * np.random.default_rng(seed).random(n ** 3))
    return box_workload("t", "elasticity", (n,) * 3, [uniform_cuts(n, n_sub)] * 3, young=young)


def test_noalloc_schur_matches_apply_schur():
    from paper_1201_5991_amd import Problem, Solver
    print("[no-alloc] S^ through the static scratch", flush=True)
    for prob_w, seed in ((_cube(4, 6, 1), 11), (_cube(2, 3, 2), 12)):   # the second call is smaller
        s = Solver(use_graph=False).setup(Problem(prob_w))
        x = torch.tensor(np.random.default_rng(seed).standard_normal(s.n_iface), device="cuda")
        y_ref = s.apply_schur(x)
        y = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        st = s.lib.mlbddc_apply_schur_noalloc(s.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
        torch.cuda.synchronize()
        assert st == 0, st
        assert torch.cuda.memory_allocated() == before
        err = float(torch.linalg.norm(y - y_ref) / torch.linalg.norm(y_ref))
        print(f"  n_iface {s.n_iface}: rel diff vs mlbddc_apply_schur {err:.2e}", flush=True)
        assert err < 1e-10
        s.destroy()

"""Failure paths and the device allocator, through the C ABI (runs on an MI355X).

Every case ends with a status returned to the host; no kernel is made to
fault or hang:
* E_NOT_CONVERGED: PCG stopped by max_iter; u holds the last iterate, which
  equals the oracle's iterate after the same number of iterations (the PCG
  iterates are unique in exact arithmetic) to relative 1e-10;
* E_BREAKDOWN: a non-finite right-hand side gives p^T S p not finite; no
  step is taken;
* E_SINGULAR_CONSTRAINTS: with corner constraints only, an interface node
  whose elements in one subdomain all have zero modulus gives that
  subdomain's constrained problem an exactly zero row;
* the device memory of a handle comes from torch's caching allocator and
  goes back to it on destroy.
"""

import gc

import numpy as np
import pytest
import torch

from oracle import fem
from oracle.bddc import MultilevelBDDC
from oracle.krylov import pcg
from workloads import box_workload
from workloads.gen import uniform_cuts

pytestmark = pytest.mark.gpu


def _cube(n_sub, el, groups=(), young=None, constraints="cef"):
    n = n_sub * el
    return box_workload("t", "elasticity", (n,) * 3, [uniform_cuts(n, n_sub)] * 3, groups=groups, young=young,
                        constraints=constraints)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_not_converged_returns_last_iterate(precision):
    from paper_1201_5991_amd import MlbddcError, Problem, Solver
    print(f"[failures] not converged, {precision}", flush=True)
    w = _cube(3, 4, groups=(), young=10 ** (2 * np.random.default_rng(3).random(12 ** 3)))
    b = MultilevelBDDC(w)
    _, f = fem.assemble_global(w)
    k = 3
    s = Solver(precision=precision, max_iter=k, use_graph=True).setup(Problem(w))
    ft = torch.tensor(f, device="cuda")
    with pytest.raises(MlbddcError) as ex:
        s.solve(ft)
    assert ex.value.name == "E_NOT_CONVERGED"
    u, st = s.solve(ft, raise_on_error=False)
    assert st["status"] == "E_NOT_CONVERGED" and st["iterations"] == k and st["converged"] == 0
    ref = pcg(b.schur_apply, b.condense(f), b.apply, tol=0.0, max_iter=k)
    uh = u.cpu().numpy()[b.level1.iface_dofs]
    err = _rel(uh, ref.x)
    print(f"  iterate after {k} iterations vs oracle: {err:.2e}", flush=True)
    if precision == "fp64":
        assert err < 1e-10
        assert _rel(u.cpu().numpy(), b.recover(f, ref.x)) < 1e-10
        assert abs(st["rel_res"] - ref.rel_res) < 1e-8 * ref.rel_res
    else:
        assert err < 1e-4


def test_breakdown_on_nonfinite_rhs():
    from paper_1201_5991_amd import Problem, Solver
    print("[failures] breakdown", flush=True)
    w = _cube(2, 4)
    prob = Problem(w)
    s = Solver(use_graph=True).setup(prob)
    f = torch.tensor(prob.load_vector(), device="cuda")
    f[5] = float("nan")
    u, st = s.solve(f, raise_on_error=False)
    assert st["status"] == "E_BREAKDOWN" and st["converged"] == 0
    # the handle stays usable: a finite right-hand side solves afterwards
    u2, st2 = s.solve(torch.tensor(prob.load_vector(), device="cuda"))
    assert st2["status"] == "OK" and st2["converged"] == 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_singular_constraints(precision):
    from paper_1201_5991_amd import MlbddcError, Problem, Solver
    print(f"[failures] singular constrained problem, {precision}", flush=True)
    n_sub, el = 2, 4
    w = _cube(n_sub, el, constraints="c")
    # the four elements of subdomain 0 around the face node (el, 1, 1) (a face
    # node shared with subdomain 1, not a corner) get zero modulus
    young = np.ones(w.n_elems)
    n = n_sub * el
    for dz in (0, 1):
        for dy in (0, 1):
            young[(el - 1) + n * (dy + n * dz)] = 0.0
    w.young = young
    with pytest.raises(MlbddcError) as ex:
        Solver(precision=precision).setup(Problem(w))
    assert ex.value.name == "E_SINGULAR_CONSTRAINTS"
    assert ex.value.info.level == 1 and ex.value.info.subdomain == 0


def test_device_memory_from_torch_allocator():
    from paper_1201_5991_amd import Problem, Solver
    print("[allocator]", flush=True)
    w = _cube(3, 4)
    prob = Problem(w)
    gc.collect()           # handles of earlier tests left in reference cycles release their blocks now, not mid-test
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = Solver(use_graph=True).setup(prob)
    torch.cuda.synchronize()
    during = torch.cuda.memory_allocated()
    assert during - before > 1 << 20, (before, during)
    u, st = s.solve(torch.tensor(prob.load_vector(), device="cuda"))
    assert st["converged"] == 1
    del u
    s.setup(prob)          # a second set-up of the same problem reuses the blocks
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == during
    s.destroy()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before

"""GPU checks of the differentiable solve (runs on an MI355X).

BDDCSolve.forward sets E_e = exp(theta_e) and solves K u = f with the
multilevel BDDC-PCG; backward solves the adjoint system with the same set-up
and forms dJ/dtheta_e = -lambda_e^T (dK_e/dtheta_e) u_e in the library.  For
the compliance J = f^T u the checks are:

* the identity sum_e dJ/dtheta_e = -J (scaling every modulus by e^t scales
  u by e^-t);
* the oracle's direct-solve gradient (sparse LU of the global matrix) on a
  reduced instance of the differentiation workload's shape (32^3 elements,
  64 subdomains of 8^3, 3 levels), stored by tests/golden/make_golden.py;
* at full size (64^3, 512 subdomains of 8^3, 3 levels, 262,144 moduli) the
  oracle's gradient from its own BDDC-PCG at rtol 1e-12 (stored likewise),
  and central finite differences (h = 1e-3) of GPU solves on the 20 seeded
  elements the fixture lists;
* a small case against a direct solve computed in the test.
"""

import json
import os

import numpy as np
import pytest
import torch

from oracle.direct import direct_solve
from oracle.grad import compliance_gradient
from workloads import box_workload, config
from workloads.gen import uniform_cuts

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _load(name):
    path = os.path.join(HERE, "golden", f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def _reduced_workload():
    n = 32 ** 3
    theta = np.random.default_rng(0).normal(0.0, 0.5, n)
    return box_workload("elasticity3d_32cube_64sub_L3_grad", "elasticity", (32,) * 3, [uniform_cuts(32, 4)] * 3,
                        groups=[(2, 2, 2)], young=np.exp(theta)), theta


def _grad(w, theta0, rtol=1e-12):
    from paper_1201_5991_amd import BDDCSolve, Problem, Solver
    prob = Problem(w)
    s = Solver(rtol=rtol, use_graph=True).setup(prob)
    f = torch.tensor(prob.load_vector(), device="cuda")
    theta = torch.tensor(theta0, device="cuda", requires_grad=True)
    u = BDDCSolve.apply(theta, f, s)
    J = torch.dot(f, u)
    J.backward()
    return s, f, J.item(), theta.grad.cpu().numpy()


def _fd(s, f, theta0, elems, h=1e-3):
    from paper_1201_5991_amd import BDDCSolve
    out = []
    for e in elems:
        vals = []
        for sgn in (1.0, -1.0):
            t = theta0.copy()
            t[e] += sgn * h
            with torch.no_grad():
                up = BDDCSolve.apply(torch.tensor(t, device="cuda"), f, s)
            vals.append(torch.dot(f, up).item())
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.asarray(out)


def test_gradient_reduced_vs_direct_solve():
    print("[grad] 32^3 reduced instance vs oracle direct-solve gradient", flush=True)
    gold = _load("elasticity32_grad_L3")
    w, theta0 = _reduced_workload()
    s, f, J, g = _grad(w, theta0)
    idx = np.asarray(gold["sample_idx"])
    assert abs(J - gold["J"]) < 1e-10 * abs(gold["J"])
    err = np.abs(g[idx] - np.asarray(gold["grad_samples"])).max() / gold["grad_absmax"]
    print(f"  J {J:.12e} (oracle {gold['J']:.12e}); gradient samples rel err {err:.2e}", flush=True)
    assert err < 1e-8
    assert abs(np.linalg.norm(g) - gold["grad_norm"]) < 1e-8 * gold["grad_norm"]
    assert abs(g.sum() + J) < 1e-9 * abs(J)
    fdi = np.asarray(gold["fd_idx"])
    assert np.abs(g[fdi] - np.asarray(gold["grad_fd_elems"])).max() < 1e-8 * gold["grad_absmax"]


def test_gradient_fullsize_fd_and_oracle():
    print("[grad] 64^3 differentiation workload: oracle BDDC-PCG gradient, FD on 20 elements", flush=True)
    gold = _load("elasticity64_grad_L3")
    w = config(5)
    theta0 = np.random.default_rng(w.seed).normal(0.0, 0.5, w.n_elems)   # the workload's own field
    assert np.array_equal(np.exp(theta0), w.young)
    s, f, J, g = _grad(w, theta0)
    assert g.shape == (64 ** 3,)
    assert abs(J - gold["J"]) < 1e-9 * abs(gold["J"])
    idx = np.asarray(gold["sample_idx"])
    err = np.abs(g[idx] - np.asarray(gold["grad_samples"])).max() / gold["grad_absmax"]
    print(f"  J {J:.12e} (oracle {gold['J']:.12e}); gradient samples rel err {err:.2e}", flush=True)
    assert err < 1e-7
    assert abs(g.sum() + J) < 1e-9 * abs(J)
    fdi = np.asarray(gold["fd_idx"])
    assert len(fdi) == 20
    fd = _fd(s, f, theta0, fdi)
    fd_err = np.abs(fd - g[fdi]).max() / np.abs(g[fdi]).max()
    print(f"  central FD on 20 elements vs adjoint: max rel err {fd_err:.2e}", flush=True)
    assert np.all(np.abs(fd - g[fdi]) < 1e-5 * np.abs(g).max() + 1e-5 * np.abs(g[fdi]))
    assert np.abs(g[fdi] - np.asarray(gold["grad_fd_elems"])).max() < 1e-7 * gold["grad_absmax"]


def test_autograd_gradient_small():
    from paper_1201_5991_amd import Problem
    print("[grad] 12^3 vs direct solve", flush=True)
    rng = np.random.default_rng(11)
    theta0 = rng.normal(0.0, 0.5, 12 ** 3)
    w = box_workload("grad", "elasticity", (12, 12, 12), [uniform_cuts(12, 4)] * 3, groups=[(2, 2, 2)],
                     young=np.exp(theta0))
    s, f, J, g = _grad(w, theta0)
    ud, _, fd = direct_solve(w)
    gd = compliance_gradient(w, ud, ud)
    assert abs(J - fd @ ud) < 1e-10 * abs(fd @ ud)
    assert np.linalg.norm(g - gd) < 1e-8 * np.linalg.norm(gd)
    assert abs(g.sum() + J) < 1e-9 * abs(J)
    elems = rng.choice(12 ** 3, 4, replace=False)
    fdv = _fd(s, f, theta0, elems)
    assert np.all(np.abs(fdv - g[elems]) < 1e-5 * np.abs(g).max() + 1e-6 * np.abs(g[elems]))

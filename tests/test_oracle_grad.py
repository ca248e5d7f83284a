"""Pins of the oracle's compliance gradient (CPU only).

J = f^T u is self-adjoint (the adjoint solution equals u) and homogeneous of
degree -1 in the moduli, so sum_e dJ/dtheta_e = -J exactly; central finite
differences give the remaining entries.
"""

import numpy as np

from oracle import fem
from oracle.direct import direct_solve, solve_bddc
from oracle.grad import compliance_gradient, element_energy
from workloads import box_workload
from workloads.gen import uniform_cuts


def _wl(theta):
    return box_workload("t", "elasticity", (6, 6, 6), [uniform_cuts(6, 2)] * 3, young=np.exp(theta))


def test_gradient_sum_and_fd():
    rng = np.random.default_rng(0)
    theta = rng.normal(0.0, 0.5, 216)
    w = _wl(theta)
    u, K, f = direct_solve(w)
    J = f @ u
    g = compliance_gradient(w, u, u)
    assert np.isclose(g.sum(), -J, rtol=1e-12)
    # element energies assemble back to the global energy: sum_e E_e u_e^T K_e^0 u_e = u^T K u
    assert np.isclose(element_energy(w, u, u).sum(), u @ K @ u, rtol=1e-12)
    h = 1e-4
    for e in rng.choice(216, 6, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h; tm[e] -= h
        up, _, fp = direct_solve(_wl(tp)); um, _, fm = direct_solve(_wl(tm))
        fd = (fp @ up - fm @ um) / (2 * h)
        assert abs(fd - g[e]) < 1e-6 * abs(g).max()


def test_bddc_adjoint_equals_direct():
    rng = np.random.default_rng(1)
    w = _wl(rng.normal(0.0, 0.5, 216))
    u, res, b, f = solve_bddc(w, n_levels=2, tol=1e-12)
    ud, _, _ = direct_solve(w)
    g = compliance_gradient(w, u, u)
    gd = compliance_gradient(w, ud, ud)
    assert np.abs(g - gd).max() < 1e-9 * np.abs(gd).max()

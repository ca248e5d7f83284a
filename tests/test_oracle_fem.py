"""Pins of the oracle's FE discretisation against closed forms (CPU only).

The paper's own discretisations are not reproducible here (its meshes are not
available), so the FE layer is pinned to calculus and elasticity theory:
exact energies of polynomial fields, rigid-body null spaces, the patch test,
total loads and a Fourier-series solution of the Poisson problem.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from oracle.direct import direct_solve
from workloads import box_workload
from workloads.gen import uniform_cuts


def test_q1_energies_of_polynomial_fields():
    # Energy int |grad u|^2 over the square [0,h]^2 for fields in the Q1 space.
    K = fem.q1_laplace_element()
    h = 0.37
    xy = np.array([[0, 0], [h, 0], [h, h], [0, h]])
    x, y = xy[:, 0], xy[:, 1]
    assert np.allclose(K @ np.ones(4), 0.0)                  # constants carry no energy
    assert np.isclose(x @ K @ x, h * h)                     # |grad x|^2 = 1 over area h^2
    assert np.isclose(y @ K @ y, h * h)
    assert np.isclose(x @ K @ y, 0.0)                        # grad x . grad y = 0
    u = x * y                                                # int (y^2 + x^2) = 2 h^4 / 3
    assert np.isclose(u @ K @ u, 2 * h ** 4 / 3)
    assert np.isclose(u @ K @ x, h ** 3 / 2)                 # int y = h^3 / 2
    assert np.allclose(K, K.T)


def _rigid_modes():
    X = fem.HEX_NODES * 0.5 + 0.5   # unit cube coordinates of the 8 nodes
    modes = []
    for c in range(3):
        t = np.zeros((8, 3)); t[:, c] = 1.0
        modes.append(t.ravel())
    for axis in range(3):
        w = np.zeros(3); w[axis] = 1.0
        modes.append(np.cross(w, X).ravel())
    return np.array(modes).T


@pytest.mark.parametrize("nu", [0.3, 0.45])
def test_hex8_null_space_and_rank(nu):
    K = fem.hex8_elasticity_element(1.0, nu, 1.0)
    assert np.allclose(K, K.T, atol=1e-14)
    assert np.abs(K @ _rigid_modes()).max() < 1e-12
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12
    assert np.sum(ev > 1e-10 * ev[-1]) == 18      # full integration: no hourglass modes


def test_hex8_uniform_strain_energies():
    # For a linear field u = eps x the element energy is vol * e^T D e (Voigt,
    # engineering shears).  E = 1, nu = 0.3 gives lambda = 0.5769230769...,
    # mu = 0.3846153846..., bulk modulus 0.8333...
    lam, mu = 0.3 / (1.3 * 0.4), 1.0 / 2.6
    assert np.isclose(lam, 0.576923076923077) and np.isclose(mu, 0.384615384615385)
    h = 0.25
    K = fem.hex8_elasticity_element(1.0, 0.3, h)
    X = (fem.HEX_NODES * 0.5 + 0.5) * h
    vol = h ** 3

    def field(F):
        return (X @ F.T).ravel()

    uni = field(np.diag([1.0, 0, 0]))
    assert np.isclose(uni @ K @ uni, vol * (lam + 2 * mu))
    shear = field(np.array([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]]))  # u_x = y: gamma_xy = 1
    assert np.isclose(shear @ K @ shear, vol * mu)
    hydro = field(np.eye(3))
    assert np.isclose(hydro @ K @ hydro, vol * 9 * (1.0 / (3 * (1 - 0.6))))
    assert np.isclose(K.sum(), 0.0, atol=1e-12)


def test_total_load_unit_body_force():
    w = box_workload("t", "elasticity", (6, 6, 6), [uniform_cuts(6, 2)] * 3)
    assert np.allclose(fem.total_load(w), [0.0, 0.0, -1.0])
    w2 = box_workload("t", "poisson", (8, 8), [uniform_cuts(8, 2)] * 2, dirichlet="all")
    assert np.isclose(fem.total_load(w2)[0], 1.0)


def test_elasticity_patch_test():
    # A linear displacement imposed on the whole boundary of a homogeneous body,
    # no body force: the interior nodes must reproduce it exactly.
    w = box_workload("t", "elasticity", (4, 4, 4), [uniform_cuts(4, 2)] * 3, body_force=(0.0, 0.0, 0.0),
                     young=np.full(64, 2.5))
    w.dirichlet_nodes[:] = False          # assemble on all DOFs
    Kall, f = fem.assemble_global(w)
    assert np.abs(f).max() == 0.0
    n1 = 5
    idx = np.arange(n1 ** 3)
    coords = np.stack([idx % n1, (idx // n1) % n1, idx // (n1 * n1)], axis=1) / 4.0
    F = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [0.2, 0.1, -0.15]])
    u_lin = (coords @ F.T + np.array([0.01, -0.02, 0.03])).ravel()
    bnd = np.any((coords == 0) | (coords == 1), axis=1)
    free = np.repeat(~bnd, 3)
    Kff = Kall[free][:, free].tocsc()
    rhs = -(Kall[free][:, ~free] @ u_lin[~free])
    u_in = spla.spsolve(Kff, rhs)
    assert np.abs(u_in - u_lin[free]).max() < 1e-12


def _series_center(terms=401):
    s = 0.0
    for m in range(1, terms, 2):
        for n in range(1, terms, 2):
            s += 16.0 / (np.pi ** 4 * m * n * (m * m + n * n)) * np.sin(m * np.pi / 2) * np.sin(n * np.pi / 2)
    return s


def test_poisson_converges_to_fourier_series():
    # -Lap u = 1 on the unit square with u = 0 on the boundary has the double sine series
    # u = sum_{m,n odd} 16 / (pi^4 m n (m^2+n^2)) sin(m pi x) sin(n pi y).
    exact = _series_center()
    errs = []
    for n in (8, 16, 32):
        w = box_workload("t", "poisson", (n, n), [uniform_cuts(n, 2)] * 2, dirichlet="all")
        u, _, _ = direct_solve(w)
        node_to_free, _ = fem.dof_numbering(w)
        centre = (n // 2) + (n + 1) * (n // 2)
        errs.append(abs(u[node_to_free[centre]] - exact))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 2e-4
    assert np.all(rates > 1.8)          # second order nodal convergence

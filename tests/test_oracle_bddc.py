"""Pins of the oracle's decomposition, preconditioner and Krylov layer (CPU only).

Each test checks the oracle against something other than itself: closed-form
glob counts of box partitions, algebraic identities of Eq. (1), the exact
preconditioner obtained when every interface DOF is primal, the BDDC spectral
lower bound lambda_min(M S) >= 1, dense eigenvalues, direct solves, and the
condition-number trend with H/h and with the number of levels (section 2).
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from oracle.bddc import MultilevelBDDC
from oracle.direct import direct_solve, solve_bddc
from oracle.krylov import lanczos_extremes, pcg
from workloads import box_workload, config
from workloads.gen import uniform_cuts

from nonbox import nonbox as _nonbox, ring_2d as _ring_2d


def cube(n_sub, el_per_sub, groups=(), young=None, **kw):
    n = n_sub * el_per_sub
    return box_workload("t", "elasticity", (n,) * 3, [uniform_cuts(n, n_sub)] * 3, groups=groups,
                        young=young, **kw)


# ----------------------------------------------------------------------------- globs
@pytest.mark.parametrize("n", [2, 3])
def test_glob_counts_3d_closed_form(n):
    # n x n x n boxes with one clamped face: interior cross points (n-1)^3 corners,
    # 3 n (n-1)^2 edge segments and 3 n^2 (n-1) face patches.
    w = cube(n, 3)
    b = MultilevelBDDC(w, n_levels=2)
    c = b.level1.glob_counts()
    assert c == {"corner": (n - 1) ** 3, "edge": 3 * n * (n - 1) ** 2, "face": 3 * n * n * (n - 1)}
    assert b.level1.n_coarse == 3 * sum(c.values())


def test_glob_counts_2d_closed_form():
    # 4 x 4 squares, whole boundary Dirichlet: 9 cross points, 2*4*3 = 24 edges;
    # corners-only coarse space of size 9.
    b = MultilevelBDDC(config(1))
    assert b.level1.glob_counts() == {"corner": 9, "edge": 24, "face": 0}
    assert b.coarse_sizes() == [9]
    assert b.level1.n_iface == 177


def test_level_two_glob_counts():
    # 4^3 boxes grouped 2x2x2: the level-2 pseudo-mesh is 2^3 subdomains whose
    # interface has 1 corner, 6 edges and 12 faces -> top coarse size 57.
    b = MultilevelBDDC(cube(4, 3, groups=[(2, 2, 2)]), n_levels=3)
    assert b.levels[1].glob_counts() == {"corner": 1, "edge": 6, "face": 12}
    assert b.coarse_sizes() == [837, 57]


# -------------------------------------------------------------------------- weights
@pytest.mark.parametrize("weights", ["stiffness", "multiplicity"])
def test_weights_partition_of_unity(weights):
    rng = np.random.default_rng(3)
    w = cube(2, 3, young=10 ** (3 * rng.random(216)))
    lev = MultilevelBDDC(w, n_levels=2, weights=weights).level1
    s = np.zeros(lev.n_iface)
    for i in range(lev.n_sub):
        np.add.at(s, lev.R[i], lev.D[i])
    assert np.allclose(s, 1.0, atol=1e-14)


def test_stiffness_weights_two_materials():
    # Two 2D subdomains with moduli 1 and 3: the diagonal of each interface node
    # scales with the modulus, so the weights are 1/4 and 3/4.
    young = np.where(np.arange(16) % 4 < 2, 1.0, 3.0)
    w = box_workload("t", "poisson", (4, 4), [uniform_cuts(4, 2), [0, 4]], young=young, dirichlet="all")
    lev = MultilevelBDDC(w, n_levels=2).level1
    assert lev.n_iface == 3
    assert np.allclose(lev.D[0], 0.25) and np.allclose(lev.D[1], 0.75)


def test_stiffness_equals_multiplicity_homogeneous():
    w = cube(3, 3)
    a = MultilevelBDDC(w, n_levels=2, weights="stiffness").level1
    b = MultilevelBDDC(w, n_levels=2, weights="multiplicity").level1
    for i in range(a.n_sub):
        assert np.allclose(a.D[i], b.D[i], atol=1e-14)


# ----------------------------------------------------------------- coarse basis (1)
def test_coarse_basis_identities():
    rng = np.random.default_rng(0)
    w = cube(3, 3, young=10 ** (3 * rng.random(729)))
    lev = MultilevelBDDC(w, n_levels=2).level1
    for i in range(lev.n_sub):
        K, C, Psi, Lam = lev.K[i].toarray(), lev.C[i].toarray(), lev.Psi[i], lev.Lam[i]
        assert np.allclose(C @ Psi, np.eye(C.shape[0]), atol=1e-10)              # constraints hold
        assert np.allclose(Psi.T @ K @ Psi, -Lam, rtol=1e-9, atol=1e-9 * np.abs(Lam).max())  # K_Ci = -Lambda_i
        # energy minimality: K Psi is orthogonal to the null space of C
        N = np.linalg.svd(C)[2][C.shape[0]:].T
        assert np.abs(N.T @ K @ Psi).max() < 1e-9 * np.abs(K).max()
    ev = np.linalg.eigvalsh(lev.KC)
    assert ev[0] > 0                                                                  # K_C is SPD


# -------------------------------------------------------------- interface problem
def test_interface_problem_matches_direct_solve():
    rng = np.random.default_rng(1)
    w = cube(2, 4, young=10 ** (3 * rng.random(512)))
    b = MultilevelBDDC(w, n_levels=2)
    u, K, f = direct_solve(w)
    lev = b.level1
    g = b.condense(f)
    u_hat = u[lev.iface_dofs]
    assert np.linalg.norm(b.schur_apply(u_hat) - g) < 1e-10 * np.linalg.norm(g)
    assert np.allclose(b.recover(f, u_hat), u, rtol=0, atol=1e-11 * np.abs(u).max())


def test_schur_is_spd_cfg1():
    b = MultilevelBDDC(config(1))
    lev = b.level1
    S = np.column_stack([b.schur_apply(e) for e in np.eye(lev.n_iface)])
    assert np.allclose(S, S.T, atol=1e-12)
    assert np.linalg.eigvalsh(S)[0] > 0


# ------------------------------------------------------------- preconditioner (2)
def test_all_primal_gives_one_iteration():
    # Every interface DOF a corner: the coarse problem is the whole interface
    # Schur complement and M = S^{-1}; PCG stops after one iteration.
    rng = np.random.default_rng(2)
    w = cube(2, 3, young=10 ** (2 * rng.random(216)))
    b = MultilevelBDDC(w, n_levels=2, constraints=["primal"])
    _, f = fem.assemble_global(w)
    g = b.condense(f)
    res = pcg(b.schur_apply, g, b.apply, tol=1e-12)
    assert res.iterations == 1 and res.rel_res < 1e-11


def test_dense_spectrum_cfg1_matches_lanczos():
    b = MultilevelBDDC(config(1))
    n = b.level1.n_iface
    S = np.column_stack([b.schur_apply(e) for e in np.eye(n)])
    M = np.column_stack([b.apply(e) for e in np.eye(n)])
    assert np.allclose(M, M.T, atol=1e-12)                                  # M symmetric
    ev = np.sort(np.linalg.eigvals(M @ S).real)
    assert ev[0] > 1 - 1e-10                                                 # BDDC lower bound
    _, f = fem.assemble_global(config(1))
    res = pcg(b.schur_apply, b.condense(f), b.apply, tol=1e-14, max_iter=200)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    assert lo >= ev[0] - 1e-8 and hi <= ev[-1] + 1e-8                      # Ritz values inside
    assert abs(hi - ev[-1]) < 1e-6 * ev[-1]


@pytest.mark.parametrize("L", [2, 3])
def test_lanczos_lower_bound_and_direct_agreement(L):
    rng = np.random.default_rng(4)
    w = cube(4, 3, groups=[(2, 2, 2)], young=10 ** (3 * rng.random(12 ** 3)))
    u, res, b, f = solve_bddc(w, n_levels=L, tol=1e-10)
    assert res.converged
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    assert lo > 1 - 1e-8
    ud, _, _ = direct_solve(w)
    kappa = hi / lo
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 10 * kappa * 1e-10


def test_three_level_with_primal_level_two_equals_two_level():
    w = cube(4, 3, groups=[(2, 2, 2)])
    b2 = MultilevelBDDC(w, n_levels=2)
    b3 = MultilevelBDDC(w, n_levels=3, constraints=["cef", "primal"])
    r = np.random.default_rng(5).standard_normal(b2.level1.n_iface)
    z2, z3 = b2.apply(r), b3.apply(r)
    assert np.linalg.norm(z3 - z2) < 1e-11 * np.linalg.norm(z2)


def test_condition_grows_with_levels():
    # Table 1 trend: each added level worsens the condition number.
    w = cube(4, 3, groups=[(2, 2, 2)])
    kap = []
    for L in (2, 3):
        _, res, _, _ = solve_bddc(w, n_levels=L, tol=1e-12)
        lo, hi = lanczos_extremes(res.alphas, res.betas)
        kap.append(hi / lo)
    assert kap[0] < kap[1]


def test_four_levels_bound_and_trend():
    # L = 2, 3, 4 on 8^3 subdomains grouped 2x2x2 twice (512 / 64 / 8 / 1, the
    # paper's 8:1 ratio between levels): lambda_min >= 1 at every depth (the
    # spectrum of the multilevel operator stays above the exact one), kappa
    # grows with every added level (Table 1 trend), and the solution agrees
    # with the direct solve.
    rng = np.random.default_rng(6)
    w = cube(8, 2, groups=[(2, 2, 2), (2, 2, 2)], young=10 ** (2 * rng.random(16 ** 3)))
    ud, _, _ = direct_solve(w)
    kap = []
    for L in (2, 3, 4):
        u, res, b, _ = solve_bddc(w, n_levels=L, tol=1e-12)
        assert res.converged
        lo, hi = lanczos_extremes(res.alphas, res.betas)
        assert lo > 1 - 1e-8
        kap.append(hi / lo)
        assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 10 * kap[-1] * 1e-12
    assert b.coarse_sizes() == [8589, 837, 57]
    assert kap[0] < kap[1] < kap[2]


def test_four_level_with_primal_level_three_equals_three_level():
    # making every level-3 interface node primal turns level 3 into an exact
    # solve of the level-3 problem: the 4-level preconditioner is then the
    # 3-level one, to rounding
    w = cube(8, 2, groups=[(2, 2, 2), (2, 2, 2)])
    b3 = MultilevelBDDC(w, n_levels=3)
    b4 = MultilevelBDDC(w, n_levels=4, constraints=["cef", "cef", "primal"])
    r = np.random.default_rng(7).standard_normal(b3.level1.n_iface)
    z3, z4 = b3.apply(r), b4.apply(r)
    assert np.linalg.norm(z4 - z3) < 1e-11 * np.linalg.norm(z3)


def test_condition_grows_with_H_over_h_2d():
    # The bound C (1 + log(H/h))^2: kappa increases with H/h, slower than H/h.
    kap = []
    for m in (4, 8, 16):
        w = box_workload("t", "poisson", (4 * m, 4 * m), [uniform_cuts(4 * m, 4)] * 2, dirichlet="all", constraints="c")
        _, res, _, _ = solve_bddc(w, tol=1e-12)
        lo, hi = lanczos_extremes(res.alphas, res.betas)
        assert lo > 1 - 1e-8
        kap.append(hi / lo)
    assert kap[0] < kap[1] < kap[2]
    bound = [(1 + np.log(m)) ** 2 for m in (4, 8, 16)]
    assert kap[2] / kap[0] < 1.5 * bound[2] / bound[0]


# ------------------------------------------------------------------------- Krylov
def test_pcg_identity_is_textbook_cg():
    rng = np.random.default_rng(6)
    Q = np.linalg.qr(rng.standard_normal((40, 40)))[0]
    A = Q @ np.diag(np.linspace(1, 50, 40)) @ Q.T
    b = rng.standard_normal(40)
    res = pcg(lambda v: A @ v, b, tol=1e-12, max_iter=200)
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x) < 1e-10 * np.linalg.norm(x)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    assert abs(lo - 1) < 1e-8 and abs(hi - 50) < 1e-8
    # k-th iterate of CG lies in the Krylov space and minimises the A-norm error there
    res3 = pcg(lambda v: A @ v, b, tol=0.0, max_iter=3)
    Kry = np.column_stack([b, A @ b, A @ A @ b])
    y = np.linalg.solve(Kry.T @ A @ Kry, Kry.T @ b)
    assert np.allclose(res3.x, Kry @ y, atol=1e-10)


# ---------------------------------------------------------------- non-box partitions

def test_glob_split_closed_form_2d():
    # Hand count (interior nodes (i, j), 1 <= i <= 7, 1 <= j <= 5): {A,Y} at
    # (1,2), (1,4); {A,B,Y} at (2,2), (2,4); {A,B} at (3,2), (3,4); {A,B,X} at
    # (4,2), (4,4); {A,X} the chain (5,2)-(6,2)-(6,3)-(6,4)-(5,4); {Y,B} (2,3);
    # {B,X} (4,3).  Split into connected parts: 4 single-node globs of three
    # subdomains (corners) and 7 edges; without the split {A,B,Y} and {A,B,X}
    # would be two-node edges and there would be no corner at all.
    b = MultilevelBDDC(_ring_2d())
    lv = b.level1
    assert lv.glob_counts() == {"corner": 4, "edge": 7, "face": 0}
    assert lv.n_coarse == 4
    sizes = sorted(len(g.nodes) for g in lv.globs)
    assert sizes == [1] * 10 + [5]


def test_ring_partition_solves():
    # corners only: B and X float and are held by their corners alone
    w = _ring_2d()
    u, res, b, f = solve_bddc(w, tol=1e-12)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    assert res.converged and lo > 1 - 1e-8
    ud, _, _ = direct_solve(w)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-10


@pytest.mark.parametrize("kind,L", [("kd", 2), ("grown", 2), ("grown", 3)])
def test_nonbox_partitions_bound_and_direct_agreement(kind, L):
    # k-d (T-junction) and graph-grown level-1 divisions, graph-grown level-2
    # groups: lambda_min >= 1 and the direct solution, as on boxes
    w = _nonbox(kind, L)
    u, res, b, _ = solve_bddc(w, tol=1e-12)
    assert res.converged and b.n_levels == L
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    assert lo > 1 - 1e-8
    ud, _, _ = direct_solve(w)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 10 * (hi / lo) * 1e-12


def test_grown_partition_splits_classes():
    # the graph-grown division has subdomain pairs touching in separate
    # patches: more globs than classes of equal subdomain sets, and every glob
    # lies in one class
    b = MultilevelBDDC(_nonbox("grown", 2))
    lv = b.level1
    classes = {g.subs for g in lv.globs}
    assert len(lv.globs) > len(classes)
    for g in lv.globs:
        assert all(tuple(lv.node_subs[int(n)]) == g.subs for n in g.nodes)

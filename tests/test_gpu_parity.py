"""GPU parity of the HIP library against the FP64 oracle (runs on an MI355X).

Every check calls the library through its C ABI (the ctypes binding) and
compares, element by element, with the oracle on the same seeded inputs.
Bars (FP64 path): relative 1e-10 for single applications of S^, the
preconditioner, condensation and the coarse matrices; PCG iteration counts
within +-1 of the oracle at rel. residual 1e-8.  Mixed precision: the same
1e-8 residual with at most 15 % more iterations, and the apply error against
the FP64 oracle reported.  Sizes span several 64-wide tiles with ragged
tails (interior blocks of 81..375 DOFs, interfaces of 100..700 DOFs); box
divisions and non-box ones (k-d bisection, graph-grown subdomains and
groups, a 2D ring whose subdomains touch in separate patches).
"""

import sys

import numpy as np
import pytest
import torch

from oracle import fem
from oracle.bddc import MultilevelBDDC
from oracle.direct import direct_solve
from oracle.grad import element_energy
from oracle.krylov import pcg
from workloads import box_workload, config
from workloads.gen import uniform_cuts

from nonbox import nonbox, ring_2d

pytestmark = pytest.mark.gpu

RTOL64 = 1e-10


def _cube(n_sub, el, groups=(), young=None, seed=0):
    n = n_sub * el
    return box_workload("t", "elasticity", (n,) * 3, [uniform_cuts(n, n_sub)] * 3, groups=groups, young=young, seed=seed)


CASES = {
    "poisson2d_cfg1": lambda: config(1),
    "elast_3x3x3_of_4_hetero": lambda: _cube(3, 4, young=10 ** (3 * np.random.default_rng(7).random(12 ** 3))),
    "elast_4x4x4_of_3_L3": lambda: _cube(4, 3, groups=[(2, 2, 2)],
                                         young=10 ** (2 * np.random.default_rng(8).random(12 ** 3))),
    # 4x4x4 groups: level-2 interiors of 837 DOFs (14 tiles) and interfaces of
    # 507 (8 tiles), so the level-2 products take the multi-tile path
    "elast_8x8x8_of_2_L3_g4": lambda: _cube(8, 2, groups=[(4, 4, 4)],
                                            young=10 ** (2 * np.random.default_rng(8).random(16 ** 3))),
    # four levels: 512 / 64 / 8 / 1 (2x2x2 groups twice)
    "elast_8x8x8_of_2_L4": lambda: _cube(8, 2, groups=[(2, 2, 2), (2, 2, 2)],
                                         young=10 ** (2 * np.random.default_rng(9).random(16 ** 3))),
    # non-box divisions: subdomains touching in separate patches (globs split
    # into connected parts), k-d bisection with T-junctions, graph-grown
    # subdomains and graph-grown level-2 groups
    "ring2d_poisson_corners": ring_2d,
    "elast_kd27_L2": lambda: nonbox("kd", 2),
    "elast_grown27_L3": lambda: nonbox("grown", 3),
    "elast_grown64_16cube_L3": lambda: nonbox("grown", 3, n=16, parts=64, groups=8, seed=2),
}


# Bar of the mixed apply against the FP64 oracle: FP32 local operators give
# an error of about u_32 kappa_local (u_32 = 6e-8).  Box subdomains stay
# below 1e-4; graph-grown subdomains (staircase faces, pieces one element
# thick) with moduli over two decades reach local condition numbers of
# ~1e4, so their bar is 1e-3.
MIXED_APPLY_BAR = {"elast_grown27_L3": 1e-3, "elast_grown64_16cube_L3": 1e-3}


def _mixed_its_bound(ref_its):
    """At most 15 % more iterations than the FP64 oracle, rounded up to a
    whole iteration (an iteration count below 7 allows one more)."""
    return int(np.ceil(1.15 * ref_its))

_cache = {}


def _oracle(name, levels=None):
    key = (name, levels)
    if key not in _cache:
        w = CASES[name]()
        b = MultilevelBDDC(w, n_levels=levels)
        _cache[key] = (w, b)
    return _cache[key]


def _solver(w, precision="fp64", levels=None):
    from paper_1201_5991_amd import Problem, Solver
    s = Solver(precision=precision)
    s.setup(Problem(w, n_levels=levels))
    return s


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(CASES))
def test_schur_condense_apply_fp64(name):
    _say(f"[parity] {name} fp64")
    w, b = _oracle(name)
    s = _solver(w)
    lev = b.level1
    assert s.n_iface == lev.n_iface and s.n_dofs == b.n_free
    rng = np.random.default_rng(1)
    r = rng.standard_normal(lev.n_iface)
    y = s.apply_schur(torch.tensor(r, device="cuda")).cpu().numpy()
    assert _rel(y, b.schur_apply(r)) < RTOL64
    _, f = fem.assemble_global(w)
    g = s.condense(torch.tensor(f, device="cuda")).cpu().numpy()
    assert _rel(g, b.condense(f)) < RTOL64
    z = s.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert _rel(z, b.apply(r)) < RTOL64
    # coarse matrices of every BDDC level
    for l, lv in enumerate(b.levels):
        kc = s.coarse_matrix(l + 1)
        assert np.linalg.norm(kc - lv.KC) < RTOL64 * np.linalg.norm(lv.KC)


@pytest.mark.parametrize("name", list(CASES))
def test_solve_fp64_matches_oracle(name):
    _say(f"[solve] {name} fp64")
    w, b = _oracle(name)
    s = _solver(w)
    _, f = fem.assemble_global(w)
    u, st = s.solve(torch.tensor(f, device="cuda"))
    g = b.condense(f)
    ref = pcg(b.schur_apply, g, b.apply, tol=1e-8)
    assert st["converged"] == 1 and st["rel_res"] < 1e-8
    assert abs(st["iterations"] - ref.iterations) <= 1
    ud, _, _ = direct_solve(w)
    u = u.cpu().numpy()
    kappa = st["lambda_max"] / st["lambda_min"]
    assert st["lambda_min"] > 1 - 1e-6
    assert _rel(u, ud) < 10 * kappa * 1e-8
    # true interface residual of the returned solution
    uh = u[b.level1.iface_dofs]
    assert np.linalg.norm(g - b.schur_apply(uh)) < 1e-7 * np.linalg.norm(g)


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_precision(name):
    _say(f"[mixed] {name}")
    w, b = _oracle(name)
    s = _solver(w, precision="mixed")
    rng = np.random.default_rng(2)
    r = rng.standard_normal(b.level1.n_iface)
    z = s.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    err = _rel(z, b.apply(r))
    bar = MIXED_APPLY_BAR.get(name, 1e-4)
    _say(f"  mixed apply rel error vs FP64 oracle: {err:.3e} (bar {bar:.0e})")
    assert err < bar
    _, f = fem.assemble_global(w)
    u, st = s.solve(torch.tensor(f, device="cuda"))
    ref = pcg(b.schur_apply, b.condense(f), b.apply, tol=1e-8)
    _say(f"  mixed its {st['iterations']} vs oracle {ref.iterations}")
    assert st["converged"] == 1
    assert st["iterations"] <= _mixed_its_bound(ref.iterations)
    uh = u.cpu().numpy()[b.level1.iface_dofs]
    g = b.condense(f)
    assert np.linalg.norm(g - b.schur_apply(uh)) < 1e-7 * np.linalg.norm(g)


def test_two_level_of_three_level_case():
    _say("[parity] elast_4x4x4_of_3 at two levels")
    w, b = _oracle("elast_4x4x4_of_3_L3", levels=2)
    s = _solver(w, levels=2)
    r = np.random.default_rng(3).standard_normal(b.level1.n_iface)
    z = s.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert _rel(z, b.apply(r)) < RTOL64


def test_element_energy_matches_oracle():
    _say("[energy]")
    w, b = _oracle("elast_3x3x3_of_4_hetero")
    s = _solver(w)
    rng = np.random.default_rng(4)
    a, c = rng.standard_normal(b.n_free), rng.standard_normal(b.n_free)
    e = s.element_energy(torch.tensor(a, device="cuda"), torch.tensor(c, device="cuda")).cpu().numpy()
    assert _rel(e, element_energy(w, a, c)) < 1e-13


def test_error_paths():
    from paper_1201_5991_amd import MlbddcError, Problem, Solver
    _say("[errors]")
    s = Solver()
    with pytest.raises(MlbddcError) as ex:
        s._chk(s.lib.mlbddc_apply(s.h, None, None))
    assert ex.value.name == "E_STATE"
    w = _cube(2, 3)
    w.young = w.young.copy()
    w.young[w.elem_to_sub == 0] = -1.0       # one subdomain with a negative modulus
    with pytest.raises(MlbddcError) as ex:
        s.setup(Problem(w))
    assert ex.value.name == "E_NOT_SPD"
    assert ex.value.info.level == 1 and ex.value.info.subdomain == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision):
    """A solve whose PCG iterations replay a captured HIP graph gives the same
    iterates as the eager launches; repeated solves (several replays each, with
    eager applies and synchronizations in between) agree every time."""
    from paper_1201_5991_amd import Problem, Solver
    _say(f"[graph] {precision}")
    w, b = _oracle("elast_4x4x4_of_3_L3")
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    eager = Solver(precision=precision, use_graph=False).setup(prob)
    graph = Solver(precision=precision, use_graph=True).setup(prob)
    u0, st0 = eager.solve(f)
    r = torch.tensor(np.random.default_rng(9).standard_normal(eager.n_iface), device="cuda")
    z0 = eager.apply(r)
    for rep in range(3):
        u1, st1 = graph.solve(f)
        torch.cuda.synchronize()
        assert st1["iterations"] == st0["iterations"]
        assert torch.equal(u1, u0), f"replay {rep} differs"
        z1 = graph.apply(r)          # eager work between graph solves
        torch.cuda.synchronize()
        assert torch.equal(z1, z0)


def test_uneven_boxes_three_levels():
    """Uneven batching: a 20^3 mesh cut by seeded random planes into 4x4x4
    boxes of 3..8 elements per side (different interior / interface sizes and
    envelopes per subdomain), 3 levels, FP64 and mixed."""
    from workloads.gen import random_cuts
    from paper_1201_5991_amd import Problem, Solver
    _say("[parity] uneven boxes")
    cuts = random_cuts(3, n=20, parts=4, lo=3, hi=8)
    w = box_workload("uneven", "elasticity", (20, 20, 20), cuts, groups=[(2, 2, 2)],
                     young=10 ** (2 * np.random.default_rng(5).random(20 ** 3)))
    b = MultilevelBDDC(w)
    s = Solver().setup(Problem(w))
    r = np.random.default_rng(6).standard_normal(b.level1.n_iface)
    z = s.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert _rel(z, b.apply(r)) < RTOL64
    y = s.apply_schur(torch.tensor(r, device="cuda")).cpu().numpy()
    assert _rel(y, b.schur_apply(r)) < RTOL64
    _, f = fem.assemble_global(w)
    u, st = s.solve(torch.tensor(f, device="cuda"))
    ref = pcg(b.schur_apply, b.condense(f), b.apply, tol=1e-8)
    assert abs(st["iterations"] - ref.iterations) <= 1
    sm = Solver(precision="mixed").setup(Problem(w))
    um, stm = sm.solve(torch.tensor(f, device="cuda"))
    assert stm["converged"] == 1 and stm["iterations"] <= _mixed_its_bound(ref.iterations)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lookahead_schedule_same_result(precision):
    """The two-stream (look-ahead) factorization schedule applies the same
    tile updates in the same order per tile as the one-stream schedule, so
    both set-ups give the same operators and the same solve."""
    from paper_1201_5991_amd import Problem, Solver
    _say(f"[parity] look-ahead schedule, {precision}")
    # 2x2x2 subdomains of 8^3 elements: 17 interior tile columns, several panels of 2
    w = _cube(2, 8, young=10 ** (2 * np.random.default_rng(10).random(16 ** 3)))
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    s1 = Solver(precision=precision, lookahead=False, panel_tiles=2, panel_tiles_precond=2).setup(prob)
    s2 = Solver(precision=precision, lookahead=True, panel_tiles=2, panel_tiles_precond=2).setup(prob)
    r = torch.tensor(np.random.default_rng(9).standard_normal(s1.n_iface), device="cuda")
    assert torch.equal(s1.apply_schur(r), s2.apply_schur(r))
    assert torch.equal(s1.apply(r), s2.apply(r))
    u1, st1 = s1.solve(f)
    u2, st2 = s2.solve(f)
    assert st1["iterations"] == st2["iterations"]
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_staged_columns_same_result(precision):
    """The tile products stage 16, 32 or 64 columns per step and accumulate
    over k in the same order for each, so every choice gives bitwise the same
    operators and solve; the 32-column results also match the oracle."""
    from paper_1201_5991_amd import Problem, Solver
    _say(f"[parity] staged columns 16 / 32 / 64, {precision}")
    w = _cube(2, 8, young=10 ** (2 * np.random.default_rng(10).random(16 ** 3)))
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    r = None
    out = {}
    for stage in (16, 32, 64):
        s = Solver(precision=precision, stage_cols=stage, panel_tiles=3, panel_tiles_precond=3).setup(prob)
        assert s.profile()["jobs"]["stage_K"] == stage
        if r is None:
            r = torch.tensor(np.random.default_rng(9).standard_normal(s.n_iface), device="cuda")
        u, st = s.solve(f)
        out[stage] = (s.apply_schur(r), s.apply(r), u, st["iterations"])
        s.destroy()
    for stage in (16, 64):
        for a, b in zip(out[stage], out[32]):
            assert (a == b) if isinstance(a, int) else torch.equal(a, b), stage
    b = MultilevelBDDC(w)
    rr = r.cpu().numpy()
    assert _rel(out[32][0].cpu().numpy(), b.schur_apply(rr)) < RTOL64
    if precision == "fp64":
        assert _rel(out[32][1].cpu().numpy(), b.apply(rr)) < RTOL64


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mv_group_tiles_same_result(precision):
    """The large tile products (S^, the level-1 local operators) take one or
    two stored tiles per workgroup with the same per-tile arithmetic: the
    operators and the solve agree bitwise."""
    from paper_1201_5991_amd import Problem, Solver
    _say(f"[parity] tiles per workgroup 1 / 2, {precision}")
    # 3^3 subdomains of 8^3 elements: interface blocks of 10-19 tiles, odd tile counts per block
    w = _cube(3, 8, young=10 ** (2 * np.random.default_rng(11).random(24 ** 3)))
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    out = {}
    r = None
    for tpw in (1, 2):
        s = Solver(precision=precision, mv_group_tiles=tpw, use_graph=True).setup(prob)
        if r is None:
            r = torch.tensor(np.random.default_rng(12).standard_normal(s.n_iface), device="cuda")
        u, st = s.solve(f)
        out[tpw] = (s.apply_schur(r), s.apply(r), u, st["iterations"])
        s.destroy()
    assert out[1][3] == out[2][3]
    for a, b in zip(out[1][:3], out[2][:3]):
        assert torch.equal(a, b)
    b = MultilevelBDDC(w)
    assert _rel(out[2][0].cpu().numpy(), b.schur_apply(r.cpu().numpy())) < RTOL64


def test_mfma_shape_fp32():
    """The three forms of the FP32 tile products: 2x2 blocks of 16x16x4 MFMA
    per wavefront, one 32x32x2 block, and the split form (three bf16 pieces
    per operand, six piece products on the bf16 MFMA).  The 32x32x2
    mixed apply agrees with the 16x16x4 one to FP32 rounding (1e-5; on gfx950
    the two came out bitwise equal); the split form sums in another order
    and agrees to 1e-4, the mixed bar; each
    agrees with the FP64 oracle to the mixed bar, and each solve takes the
    same iterations within one.  FP64 factorizations do not use the form
    (bitwise the same)."""
    from paper_1201_5991_amd import Problem, Solver
    _say("[parity] FP32 tile products: 16x16x4 / 32x32x2 / split bf16")
    # 4x4x4 subdomains of 4^3 elements, 2x2x2 level-2 groups: FP32 constrained problems on both levels
    # and an FP32 level-2 K job
    w = _cube(4, 4, groups=[(2, 2, 2)], young=10 ** (2 * np.random.default_rng(13).random(16 ** 3)))
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    out = {}
    r = None
    shapes = (16, 32, 3)
    for prec in ("mixed", "fp64"):
        for sh in shapes:
            s = Solver(precision=prec, mfma_f32=sh, use_graph=True).setup(prob)
            if r is None:
                r = torch.tensor(np.random.default_rng(14).standard_normal(s.n_iface), device="cuda")
            u, st = s.solve(f)
            out[(prec, sh)] = (s.apply(r), s.apply_schur(r), u, st["iterations"])
            s.destroy()
    for sh in shapes[1:]:
        for a, b in zip(out[("fp64", 16)][:3], out[("fp64", sh)][:3]):
            assert torch.equal(a, b)
    b = MultilevelBDDC(w)
    ref = b.apply(r.cpu().numpy())
    m16 = out[("mixed", 16)]
    for sh, bar in ((32, 1e-5), (3, 1e-4)):
        m = out[("mixed", sh)]
        assert torch.equal(m16[1], m[1])  # S^ is FP64
        err = _rel(m[0].cpu().numpy(), m16[0].cpu().numpy())
        eo = _rel(m[0].cpu().numpy(), ref)
        _say(f"  mixed apply, form {sh} against 16x16x4: {err:.2e}; against the oracle {eo:.2e}; "
             f"iterations {m[3]} / {m16[3]}")
        assert err < bar
        assert abs(m[3] - m16[3]) <= 1
        assert eo < 1e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_update_coefficients_matches_fresh_setup(precision):
    """A numeric re-set-up with new element moduli (the plan, layouts and
    schedules kept) gives bitwise the operators and solve of a set-up from
    scratch with those moduli, on dissection-ordered, tile-mapped factors."""
    from paper_1201_5991_amd import Problem, Solver
    _say(f"[parity] update_coefficients vs fresh set-up, {precision}")
    rng = np.random.default_rng(13)
    w1 = _cube(2, 8, young=10 ** (2 * rng.random(16 ** 3)))
    w2 = _cube(2, 8, young=10 ** (2 * rng.random(16 ** 3)))
    p1, p2 = Problem(w1), Problem(w2)
    f = torch.tensor(p2.load_vector(), device="cuda")
    s1 = Solver(precision=precision).setup(p1)
    s1.update_coefficients(torch.tensor(w2.young, device="cuda"))
    s2 = Solver(precision=precision).setup(p2)
    r = torch.tensor(np.random.default_rng(14).standard_normal(s1.n_iface), device="cuda")
    assert torch.equal(s1.apply_schur(r), s2.apply_schur(r))
    assert torch.equal(s1.apply(r), s2.apply(r))
    u1, st1 = s1.solve(f)
    u2, st2 = s2.solve(f)
    assert st1["iterations"] == st2["iterations"] and torch.equal(u1, u2)
    b = MultilevelBDDC(w2)
    assert _rel(s1.apply_schur(r).cpu().numpy(), b.schur_apply(r.cpu().numpy())) < RTOL64


def test_side_stream_same_result():
    """Mixed precision at 48^3 (the G product takes the side stream there):
    the level-1 G product beside the coarse levels (fork / join on a second
    stream) gives bitwise the same applies and solves as one stream, in
    eager launches and in graph replays."""
    from paper_1201_5991_amd import Problem, Solver
    _say("[parity] side-stream G product, 48^3 mixed")
    prob = Problem(config(2, levels=3))
    f = torch.tensor(prob.load_vector(), device="cuda")
    one = Solver(precision="mixed", side_stream=False, use_graph=False).setup(prob)
    r = torch.tensor(np.random.default_rng(12).standard_normal(one.n_iface), device="cuda")
    z1 = one.apply(r)
    u1, st1 = one.solve(f)
    one.destroy()
    for graph in (False, True):
        two = Solver(precision="mixed", side_stream=True, use_graph=graph).setup(prob)
        for rep in range(3):
            assert torch.equal(two.apply(r), z1), f"apply, graph={graph}, rep {rep}"
            u2, st2 = two.solve(f)
            torch.cuda.synchronize()
            assert st2["iterations"] == st1["iterations"] and torch.equal(u2, u1), f"solve, graph={graph}, rep {rep}"
        prof = two.profile()  # noqa: F841 (profiling off: no timing collected)
        two.destroy()

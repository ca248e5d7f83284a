"""Write the full-size parity fixtures from the FP64 oracle (CPU; minutes to an hour).

Usage: python tests/golden/make_golden.py [case ...]      (default: every case)

Only the oracle is called.  For each case the oracle computes, on a seeded
interface vector r ~ N(0,1) (numpy default_rng(2024)):

* M r (Algorithm 2), S^ r and the condensed right-hand side g^ (section 2);
* BDDC-PCG to rel. residual 1e-8 (iteration count, Lanczos extremes,
  the interface solution), and the iterate after a fixed number of
  iterations (the PCG iterates are unique in exact arithmetic, the stopping
  iterate may move by one);

and stores, per vector, its norm, 256 seeded sample positions and its dot
products with four seeded N(0,1) vectors (default_rng(3000 + k)): a sample
checks single entries, a projection checks every entry at once.  The wall
times of the oracle's phases and the host they ran on are recorded with
the values (the CPU baseline of the benchmark reports them).

Gradient cases store the compliance J = f^T u and dJ/dtheta_e =
-E_e u_e^T K_e^0 u_e (the compliance is self-adjoint, lambda = u) at 256
seeded elements and at the 20 elements that the finite-difference check
perturbs, with u from the oracle's BDDC-PCG at rtol 1e-12 or from a direct
sparse solve.
"""

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem  # noqa: E402
from oracle.bddc import MultilevelBDDC  # noqa: E402
from oracle.direct import direct_solve  # noqa: E402
from oracle.grad import compliance_gradient  # noqa: E402
from oracle.krylov import lanczos_extremes, pcg  # noqa: E402
from workloads import box_workload, config, large_subdomains  # noqa: E402
from workloads.gen import uniform_cuts  # noqa: E402

R_SEED = 2024
SAMPLE_SEED = 7
PROJ_SEEDS = [3000, 3001, 3002, 3003]
K_FIXED = 10          # iterations of the fixed-count PCG iterate
N_FD = 20             # elements perturbed by the finite-difference check
FD_SEED = 5

# name -> (workload factory, number of levels or None for the workload's own)
CASES = {
    "elasticity48_L2": (lambda: config(2, levels=2), None),
    "elasticity48_L3": (lambda: config(2, levels=3), None),
    "elasticity96_L3": (lambda: config(3, levels=3), None),
    "elasticity96_L4": (lambda: config(3, levels=4), None),
    "elasticity80_uneven_L3": (lambda: config(4), None),
    "elasticity40_8sub20_L2": (lambda: large_subdomains(), None),
}


def grad_reduced():
    """The differentiation workload's shape on a mesh a direct solve handles:
    32^3 elements, 4x4x4 subdomains of 8^3, 2x2x2 level-2 groups (3 levels),
    E = exp(theta), theta ~ N(0, 0.5^2) from default_rng(0)."""
    n = 32 ** 3
    theta = np.random.default_rng(0).normal(0.0, 0.5, n)
    return box_workload("elasticity3d_32cube_64sub_L3_grad", "elasticity", (32,) * 3, [uniform_cuts(32, 4)] * 3,
                        groups=[(2, 2, 2)], young=np.exp(theta))


GRAD_CASES = {
    "elasticity64_grad_L3": (lambda: config(5), "bddc"),
    "elasticity32_grad_L3": (grad_reduced, "direct"),
}


def host_info() -> dict:
    cpu = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        pass
    return {"cpu": cpu, "nproc": os.cpu_count(), "blas_threads": threads, "numpy": np.__version__}


def vec_record(v: np.ndarray, idx: np.ndarray) -> dict:
    n = len(v)
    proj = [float(np.random.default_rng(s).standard_normal(n) @ v) for s in PROJ_SEEDS]
    return {"norm": float(np.linalg.norm(v)), "samples": v[idx].tolist(), "proj": proj}


_LEVEL1 = {}   # workload name without the level count -> (level 1, its set-up seconds)


def make(name: str) -> dict:
    factory, levels = CASES[name]
    w = factory()
    key = w.name.rsplit("_L", 1)[0]
    t0 = time.perf_counter()
    if key in _LEVEL1:   # the same mesh, partition and moduli at another level count: level 1 is shared
        lv1, t_lv1 = _LEVEL1[key]
        b = MultilevelBDDC(w, n_levels=levels, level1=lv1)
        t_setup = time.perf_counter() - t0 + t_lv1
    else:
        _LEVEL1.clear()
        b = MultilevelBDDC(w, n_levels=levels)
        t_setup = time.perf_counter() - t0
        _LEVEL1[key] = (b.level1, t_setup)
    print(f"  {name}: set-up {t_setup:.1f} s, coarse {b.coarse_sizes()}", flush=True)
    n = b.level1.n_iface
    r = np.random.default_rng(R_SEED).standard_normal(n)
    ta = time.perf_counter()
    z = b.apply(r)
    t_apply = time.perf_counter() - ta
    ts = time.perf_counter()
    y = b.schur_apply(r)
    t_schur = time.perf_counter() - ts
    f = fem.load_vector(w)
    t1 = time.perf_counter()
    g = b.condense(f)
    t_cond = time.perf_counter() - t1
    t2 = time.perf_counter()
    res = pcg(b.schur_apply, g, b.apply, tol=1e-8)
    t_pcg = time.perf_counter() - t2
    t3 = time.perf_counter()
    b.recover(f, res.x)
    t_rec = time.perf_counter() - t3
    print(f"  {name}: PCG {res.iterations} its in {t_pcg:.1f} s", flush=True)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    fixed = pcg(b.schur_apply, g, b.apply, tol=0.0, max_iter=K_FIXED)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, 256, replace=False))
    levels_used = b.n_levels
    return {
        "workload": w.name, "levels": levels_used, "n_iface": int(n), "n_dofs": int(b.n_free),
        "subdomains": [int(lv.n_sub) for lv in b.levels],
        "coarse_sizes": [int(c) for c in b.coarse_sizes()],
        "globs": [lv.glob_counts() for lv in b.levels],
        "r_seed": R_SEED, "sample_idx": idx.tolist(), "proj_seeds": PROJ_SEEDS,
        "apply": vec_record(z, idx),
        "schur": vec_record(y, idx),
        "condense": vec_record(g, idx),
        "pcg": {"iterations": res.iterations, "rel_res": res.rel_res, "lambda_min": lo, "lambda_max": hi,
                "u_hat_norm": float(np.linalg.norm(res.x)), "u_hat": vec_record(res.x, idx)},
        "pcg_fixed": {"iterations": K_FIXED, "rel_res": fixed.rel_res, "u_hat": vec_record(fixed.x, idx)},
        "oracle_time_s": {"setup": t_setup, "condense": t_cond, "pcg": t_pcg, "recover": t_rec,
                          "total": t_setup + t_cond + t_pcg + t_rec, "one_apply": t_apply, "one_schur": t_schur},
        "host": host_info(),
    }


def make_grad(name: str) -> dict:
    factory, how = GRAD_CASES[name]
    w = factory()
    t0 = time.perf_counter()
    if how == "direct":
        u, _, f = direct_solve(w)
        its = None
    else:
        b = MultilevelBDDC(w)
        f = fem.load_vector(w)
        g = b.condense(f)
        res = pcg(b.schur_apply, g, b.apply, tol=1e-12)
        u = b.recover(f, res.x)
        its = res.iterations
    t = time.perf_counter() - t0
    grad = compliance_gradient(w, u, u)
    J = float(f @ u)
    ne = w.n_elems
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(ne, 256, replace=False))
    fd_idx = np.sort(np.random.default_rng(FD_SEED).choice(ne, N_FD, replace=False))
    print(f"  {name}: J = {J:.12e} ({how}, {t:.1f} s)", flush=True)
    return {
        "workload": w.name, "levels": int(w.n_levels), "n_dofs": int(len(u)), "n_elems": int(ne),
        "solution": how, "pcg_rtol": None if how == "direct" else 1e-12, "pcg_iterations": its,
        "J": J, "grad_sum": float(grad.sum()), "grad_norm": float(np.linalg.norm(grad)),
        "grad_absmax": float(np.abs(grad).max()),
        "sample_idx": idx.tolist(), "grad_samples": grad[idx].tolist(),
        "fd_seed": FD_SEED, "fd_idx": fd_idx.tolist(), "grad_fd_elems": grad[fd_idx].tolist(),
        "oracle_time_s": t, "host": host_info(),
    }


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES) + list(GRAD_CASES)
    for nm in names:
        d = make_grad(nm) if nm in GRAD_CASES else make(nm)
        path = os.path.join(HERE, f"{nm}.json")
        with open(path, "w") as fh:
            json.dump(d, fh, indent=1)
        print(path, flush=True)

"""Full-size parity on the 48^3 elasticity workload (64 subdomains, the bench
workload) against stored oracle values (runs on an MI355X).

tests/golden/elasticity48_L{2,3}.json were written by tests/golden/make_golden.py,
which calls only the FP64 oracle.  At full size the GPU results are compared on
256 seeded sample positions and in norm: M r, S^ r and g^ to relative 1e-10
(FP64 path), the PCG iteration count within +-1, and the Lanczos extremes.
"""

import json
import os

import numpy as np
import pytest
import torch

from workloads import config

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _load(levels):
    path = os.path.join(HERE, "golden", f"elasticity48_L{levels}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


@pytest.mark.parametrize("levels", [2, 3])
def test_fullsize_fp64(levels):
    from paper_1201_5991_amd import Problem, Solver
    print(f"[fullsize] L={levels}", flush=True)
    gold = _load(levels)
    prob = Problem(config(2, levels=levels))
    s = Solver(use_graph=True).setup(prob)
    assert s.n_iface == gold["n_iface"] and s.n_dofs == gold["n_dofs"]
    assert [s.coarse_size(l + 1) for l in range(levels - 1)] == gold["coarse_sizes"]
    idx = np.asarray(gold["sample_idx"])
    r = torch.tensor(np.random.default_rng(gold["r_seed"]).standard_normal(gold["n_iface"]), device="cuda")
    f = torch.tensor(prob.load_vector(), device="cuda")
    for key, vec in (("apply", s.apply(r)), ("schur", s.apply_schur(r)), ("condense", s.condense(f))):
        v = vec.cpu().numpy()
        ref = np.asarray(gold[key]["samples"])
        assert abs(np.linalg.norm(v) - gold[key]["norm"]) < 1e-10 * gold[key]["norm"], key
        assert np.abs(v[idx] - ref).max() < 1e-10 * np.abs(ref).max(), key
    u, st = s.solve(f)
    assert st["converged"] == 1 and abs(st["iterations"] - gold["pcg"]["iterations"]) <= 1
    assert abs(st["lambda_max"] - gold["pcg"]["lambda_max"]) < 1e-3 * gold["pcg"]["lambda_max"]
    assert st["lambda_min"] > 1 - 1e-6


@pytest.mark.parametrize("levels", [3])
def test_fullsize_mixed(levels):
    from paper_1201_5991_amd import Problem, Solver
    print(f"[fullsize mixed] L={levels}", flush=True)
    gold = _load(levels)
    prob = Problem(config(2, levels=levels))
    s = Solver(precision="mixed", use_graph=True).setup(prob)
    idx = np.asarray(gold["sample_idx"])
    r = torch.tensor(np.random.default_rng(gold["r_seed"]).standard_normal(gold["n_iface"]), device="cuda")
    v = s.apply(r).cpu().numpy()
    ref = np.asarray(gold["apply"]["samples"])
    err = np.abs(v[idx] - ref).max() / np.abs(ref).max()
    print(f"  mixed apply sampled rel error vs FP64 oracle: {err:.2e}", flush=True)
    assert err < 1e-3
    f = torch.tensor(prob.load_vector(), device="cuda")
    u, st = s.solve(f)
    assert st["converged"] == 1
    assert st["iterations"] <= int(np.ceil(1.15 * gold["pcg"]["iterations"])) + 1

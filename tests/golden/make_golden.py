"""Write the full-size parity fixtures from the FP64 oracle (CPU; minutes).

Usage: python tests/golden/make_golden.py [levels ...]

For the 48^3 elasticity workload (64 subdomains of 12^3, corners + edge + face
averages) at 2 and 3 levels, the oracle computes, on a seeded interface vector
r ~ N(0,1) (numpy default_rng(2024)): M r, S^ r, the condensed right-hand side
g^, and BDDC-PCG to rel. residual 1e-8 (iteration count, Lanczos extremes).
256 seeded sample positions of each vector, together with the vectors' norms,
are stored as JSON.  Only the oracle is called.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem  # noqa: E402
from oracle.bddc import MultilevelBDDC  # noqa: E402
from oracle.krylov import lanczos_extremes, pcg  # noqa: E402
from workloads import config  # noqa: E402


def make(levels: int) -> dict:
    w = config(2, levels=levels)
    t0 = time.time()
    b = MultilevelBDDC(w)
    t_setup = time.time() - t0
    n = b.level1.n_iface
    r = np.random.default_rng(2024).standard_normal(n)
    z = b.apply(r)
    y = b.schur_apply(r)
    _, f = fem.assemble_global(w)
    g = b.condense(f)
    res = pcg(b.schur_apply, g, b.apply, tol=1e-8)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    idx = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    return {
        "workload": w.name, "levels": levels, "n_iface": int(n), "n_dofs": int(b.n_free),
        "coarse_sizes": [int(c) for c in b.coarse_sizes()],
        "r_seed": 2024, "sample_idx": idx.tolist(),
        "apply": {"norm": float(np.linalg.norm(z)), "samples": z[idx].tolist()},
        "schur": {"norm": float(np.linalg.norm(y)), "samples": y[idx].tolist()},
        "condense": {"norm": float(np.linalg.norm(g)), "samples": g[idx].tolist()},
        "pcg": {"iterations": res.iterations, "rel_res": res.rel_res, "lambda_min": lo, "lambda_max": hi,
                "u_hat_norm": float(np.linalg.norm(res.x))},
        "oracle_setup_s": t_setup,
    }


if __name__ == "__main__":
    levels = [int(a) for a in sys.argv[1:]] or [2, 3]
    for L in levels:
        d = make(L)
        path = os.path.join(HERE, f"elasticity48_L{L}.json")
        with open(path, "w") as fh:
            json.dump(d, fh, indent=1)
        print(path, d["pcg"], d["coarse_sizes"], f"setup {d['oracle_setup_s']:.1f}s", flush=True)

"""Autotuner for the panel width of the batched tile factorizations.

For each workload and precision, every candidate panel width (tile columns
per panel) is run for the two kinds of factorization jobs, the subdomain
matrices (K) and the constrained local problems (M); the set-up is profiled
and the fastest width per (job kind, precision, size bucket) is written to the
tune table that the library reads at set-up:

    <K|M> <f64|f32> <ceil(log2(max tiles per side))> <panel>

Usage (on the GPU):  python -m paper_1201_5991_amd.autotune [--configs 1,2,3,4,5] [--out FILE]
"""

from __future__ import annotations

import argparse
import math
import os
import sys

CANDIDATES = (1, 2, 3, 4, 6, 8)


def _bucket(n: int) -> int:
    return max(0, math.ceil(math.log2(max(n, 1))))


def tune(configs, reps: int = 2, log=print):
    import numpy as np
    import torch
    from . import Problem, Solver
    from workloads import config

    table = {}
    for k in configs:
        w = config(k)
        prob = Problem(w)
        for prec in ("fp64", "mixed"):
            times = {}
            for p in CANDIDATES:
                s = Solver(precision=prec, panel_tiles=p, panel_tiles_precond=p, tune_table=None)
                s.setup(prob)                     # warm-up (allocations)
                best = [math.inf, math.inf]
                for _ in range(reps):
                    s.set_profiling(True)
                    s.setup(prob)
                    j = s.profile()["jobs"]
                    best[0] = min(best[0], j["K_time_s"])
                    best[1] = min(best[1], j["M_time_s"])
                s.set_profiling(False)
                nts = []
                for lev in range(1, prob.n_levels + 1):
                    sz = s.subdomain_sizes(lev)
                    nts.append(sz)
                times[p] = best
                del s
                torch.cuda.synchronize()
                log(f"config {k} {prec} panel {p}: K {best[0]*1e3:.2f} ms, M {best[1]*1e3:.2f} ms")
            # size buckets from the level-1 matrices (the dominant jobs)
            s = Solver(precision=prec, tune_table=None)
            s.setup(prob)
            sz = s.subdomain_sizes(1)
            del s
            ntK = int(max(((a + 63) // 64 + (b + 63) // 64) for a, b, _ in sz))
            ntM = int(max(2 * ((b + 63) // 64 + (c + 63) // 64) for _, b, c in sz))
            pk = min(CANDIDATES, key=lambda p: times[p][0])
            pm = min(CANDIDATES, key=lambda p: times[p][1])
            pk_prec = "f64"                       # level-1 subdomain matrices are FP64 in both modes
            pm_prec = "f32" if prec == "mixed" else "f64"
            table[("K", pk_prec, _bucket(ntK))] = pk
            table[("M", pm_prec, _bucket(ntM))] = pm
            log(f"config {k} {prec}: K bucket {_bucket(ntK)} -> {pk}, M bucket {_bucket(ntM)} -> {pm}")
    return table


def write_table(table, path):
    with open(path, "w") as fh:
        fh.write("# panel widths chosen by paper_1201_5991_amd/autotune.py on gfx950\n")
        fh.write("# job precision ceil(log2(max tiles per side)) panel\n")
        for (job, prec, b), p in sorted(table.items()):
            fh.write(f"{job} {prec} {b} {p}\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="2,3,4,5")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.txt"))
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    t = tune([int(x) for x in a.configs.split(",")], log=lambda *x: print(*x, flush=True))
    write_table(t, a.out)
    print("wrote", a.out)

"""Autotuner for the batched tile factorizations: panel width and staged columns.

For each workload and precision, every candidate pair (panel width in tile
columns per panel, columns of a tile staged per step of the MFMA tile
products) is run for the two kinds of factorization jobs, the subdomain
matrices (K) and the constrained local problems (M); the set-up is profiled
and the fastest pair per (job kind, precision, size bucket) is written to the
tune table that the library reads at set-up:

    <K|M> <f64|f32> <ceil(log2(max tiles per side))> <panel> <stage>

The staged columns do not change the results (the products accumulate in the
same order); the panel width changes only the order of independent updates.

Usage (on the GPU):  python -m paper_1201_5991_amd.autotune [--configs 2,3,4,5] [--out FILE]
"""

from __future__ import annotations

import argparse
import math
import os
import sys

CANDIDATES = (2, 3, 4, 6)        # panel widths
STAGES = (16, 32, 64)            # staged columns per step


def _bucket(n: int) -> int:
    return max(0, math.ceil(math.log2(max(n, 1))))


def tune(configs, reps: int = 2, log=print):
    """Times per (job kind, precision, size bucket) and candidate, summed over
    every workload and mode that has matrices in that bucket; the candidate
    with the smallest sum wins."""
    import torch
    from . import Problem, Solver
    from workloads import config

    agg = {}
    for k in configs:
        w = config(k)
        prob = Problem(w)
        for prec in ("fp64", "mixed"):
            s = Solver(precision=prec, tune_table=None)
            s.setup(prob)
            sz = s.subdomain_sizes(1)
            s.destroy()
            ntK = int(max(((a + 63) // 64 + (b + 63) // 64) for a, b, _ in sz))
            ntM = int(max(2 * ((b + 63) // 64 + (c + 63) // 64) for _, b, c in sz))
            keyK = ("K", "f64", _bucket(ntK))   # level-1 subdomain matrices are FP64 in both modes
            keyM = ("M", "f32" if prec == "mixed" else "f64", _bucket(ntM))
            for p in CANDIDATES:
                for sc in STAGES:
                    s = Solver(precision=prec, panel_tiles=p, panel_tiles_precond=p, stage_cols=sc, tune_table=None)
                    s.setup(prob)                     # warm-up (allocations)
                    best = [math.inf, math.inf]
                    for _ in range(reps):
                        s.set_profiling(True)
                        s.setup(prob)
                        j = s.profile()["jobs"]
                        best[0] = min(best[0], j["K_time_s"])
                        best[1] = min(best[1], j["M_time_s"])
                    s.set_profiling(False)
                    s.destroy()
                    torch.cuda.synchronize()
                    for key, t in ((keyK, best[0]), (keyM, best[1])):
                        agg.setdefault(key, {}).setdefault((p, sc), 0.0)
                        agg[key][(p, sc)] += t
                    log(f"config {k} {prec} panel {p} stage {sc}: K {best[0]*1e3:.2f} ms ({keyK[2]}), "
                        f"M {best[1]*1e3:.2f} ms ({keyM[1]} {keyM[2]})")
    table = {}
    for key, cand in agg.items():
        table[key] = min(cand, key=lambda q: cand[q])
        log(f"{' '.join(map(str, key))}: panel {table[key][0]} stage {table[key][1]} "
            f"({cand[table[key]]*1e3:.2f} ms summed; panel 4 stage 32: {cand.get((4, 32), math.nan)*1e3:.2f} ms)")
    return table


def write_table(table, path):
    with open(path, "w") as fh:
        fh.write("# panel widths and staged columns chosen by paper_1201_5991_amd/autotune.py on gfx950\n")
        fh.write("# job precision ceil(log2(max tiles per side)) panel stage\n")
        for (job, prec, b), (p, sc) in sorted(table.items()):
            fh.write(f"{job} {prec} {b} {p} {sc}\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="2,3,4,5")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.txt"))
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    t = tune([int(x) for x in a.configs.split(",")], log=lambda *x: print(*x, flush=True))
    write_table(t, a.out)
    print("wrote", a.out)

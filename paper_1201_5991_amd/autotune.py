"""Autotuner: panel width and staged columns of the batched tile
factorizations, tiles per workgroup of the tile matrix-vector products.

For each workload and precision, every candidate pair (panel width in tile
columns per panel, columns of a tile staged per step of the MFMA tile
products) is run for the two kinds of factorization jobs, the subdomain
matrices (K) and the constrained local problems (M); the set-up is profiled
and the fastest pair per (job kind, precision, size bucket) is written to the
tune table that the library reads at set-up:

    <K|M> <f64|f32> <ceil(log2(max tiles per side))> <panel> <stage>
    MV <f64|f32> 0 <tiles per workgroup of the tile matrix-vector products>
    PANEL <f64|f32> 0 <staged columns of the panel products>
    SHAPE f32 0 <MFMA shape of the FP32 tile products: 16 (16x16x4) or 32 (32x32x2)>

The staged columns do not change the results (the products accumulate in the
same order); the panel width changes only the order of independent updates.
The split-bf16 form of the FP32 tile products (mfma_f32 = 3) is faster but
less accurate, so it is not swept: a caller opts in.

Usage (on the GPU):  python -m paper_1201_5991_amd.autotune [--configs 2,3,4,5] [--out FILE]
"""

from __future__ import annotations

import argparse
import math
import os
import sys

CANDIDATES = (2, 3, 4, 6)        # panel widths
STAGES = (16, 32, 64)            # staged columns per step
MV_GROUP_TILES = (1, 2)          # stored tiles per workgroup of the tile products


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
    # tiles per workgroup of the large tile products: S^ and G products timed
    # with events, summed over the workloads, per product precision
    mv = {("MV", "f64", 0): {}, ("MV", "f32", 0): {}}
    for k in configs:
        prob = Problem(config(k))
        for prec in ("fp64", "mixed"):
            for tpw in MV_GROUP_TILES:
                s = Solver(precision=prec, mv_group_tiles=tpw, tune_table=None)
                s.setup(prob)
                r = torch.randn(s.n_iface, dtype=torch.float64, device="cuda")
                z = torch.empty_like(r)
                for _ in range(5):
                    s.apply_into(r, z)
                    s.apply_schur_into(r, z)
                s.set_profiling(True)
                for _ in range(20):
                    s.apply_schur_into(r, z)
                    s.apply_into(r, z)
                torch.cuda.synchronize()
                p = s.profile()
                s.set_profiling(False)
                s.destroy()
                t_s = p["schur_mv"]["time_s"] / max(p["schur_mv"]["launches"], 1)
                t_g = p["precond_mv"]["time_s"] / max(p["precond_mv"]["launches"], 1)
                mv[("MV", "f64", 0)][tpw] = mv[("MV", "f64", 0)].get(tpw, 0.0) + t_s
                gkey = ("MV", "f32" if prec == "mixed" else "f64", 0)
                mv[gkey][tpw] = mv[gkey].get(tpw, 0.0) + t_g
                log(f"config {k} {prec} tiles per workgroup {tpw}: S^ product {t_s*1e3:.3f} ms, "
                    f"G product {t_g*1e3:.3f} ms")
    agg.update(mv)
    # staged columns of the panel products per precision, with the panel
    # widths and staged columns chosen above: K and M job times (profiled,
    # device) of FP64 panels (both modes' K jobs, the FP64 mode's M jobs) and
    # FP32 panels (the mixed mode's M jobs), summed over the workloads
    import tempfile
    best = {key: min(cand, key=lambda q: cand[q]) for key, cand in agg.items() if key[0] != "MV"}
    pan = {("PANEL", "f64", 0): {}, ("PANEL", "f32", 0): {}}
    for ps in STAGES:
        with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as fh:
            for (job, prec, b), v in sorted(best.items()):
                fh.write(f"{job} {prec} {b} {v[0]} {v[1]}\n")
            fh.write(f"PANEL f64 0 {ps}\nPANEL f32 0 {ps}\n")
            path = fh.name
        for k in configs:
            prob = Problem(config(k))
            for prec in ("fp64", "mixed"):
                s = Solver(precision=prec, tune_table=path)
                s.setup(prob)
                t = {"K": 0.0, "M": 0.0}
                for _ in range(reps):
                    s.set_profiling(True)
                    s.setup(prob)
                    torch.cuda.synchronize()
                    j = s.profile()["jobs"]
                    s.set_profiling(False)
                    t["K"] += j["K_time_s"] / reps
                    t["M"] += j["M_time_s"] / reps
                s.destroy()
                f64 = t["K"] + (t["M"] if prec == "fp64" else 0.0)
                pan[("PANEL", "f64", 0)][ps] = pan[("PANEL", "f64", 0)].get(ps, 0.0) + f64
                if prec == "mixed":
                    pan[("PANEL", "f32", 0)][ps] = pan[("PANEL", "f32", 0)].get(ps, 0.0) + t["M"]
                log(f"config {k} {prec} panel products {ps} staged columns: K {t['K']*1e3:.2f} ms, M {t['M']*1e3:.2f} ms")
        os.unlink(path)
    agg.update(pan)
    # MFMA shape of the FP32 tile products: the mixed mode's K and M job times
    # (its FP32 jobs: the constrained problems and the K jobs above level 1)
    best_pan = {key: min(cand, key=lambda q: cand[q]) for key, cand in pan.items()}
    shp = {("SHAPE", "f32", 0): {}}
    for sh in (16, 32):
        with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as fh:
            for (job, prec, b), v in sorted(best.items()):
                fh.write(f"{job} {prec} {b} {v[0]} {v[1]}\n")
            for (job, prec, b), v in sorted(best_pan.items()):
                fh.write(f"{job} {prec} {b} {v}\n")
            fh.write(f"SHAPE f32 0 {sh}\n")
            path = fh.name
        for k in configs:
            prob = Problem(config(k))
            s = Solver(precision="mixed", tune_table=path)
            s.setup(prob)
            t = 0.0
            for _ in range(reps):
                s.set_profiling(True)
                s.setup(prob)
                torch.cuda.synchronize()
                j = s.profile()["jobs"]
                s.set_profiling(False)
                t += (j["K_time_s"] + j["M_time_s"]) / reps
            s.destroy()
            shp[("SHAPE", "f32", 0)][sh] = shp[("SHAPE", "f32", 0)].get(sh, 0.0) + t
            log(f"config {k} mixed FP32 MFMA shape {sh}: K + M {t*1e3:.2f} ms")
        os.unlink(path)
    agg.update(shp)
    table = {}
    for key, cand in agg.items():
        table[key] = min(cand, key=lambda q: cand[q])
        if key[0] in ("MV", "PANEL", "SHAPE"):
            log(f"{' '.join(map(str, key))}: {table[key]} "
                f"({', '.join(f'{q}: {v*1e3:.3f} ms' for q, v in sorted(cand.items()))} summed)")
        else:
            log(f"{' '.join(map(str, key))}: panel {table[key][0]} stage {table[key][1]} "
                f"({cand[table[key]]*1e3:.2f} ms summed; panel 4 stage 32: {cand.get((4, 32), math.nan)*1e3:.2f} ms)")
    return table


def write_table(table, path):
    with open(path, "w") as fh:
        fh.write("# panel widths and staged columns chosen by paper_1201_5991_amd/autotune.py on gfx950\n")
        fh.write("# job precision ceil(log2(max tiles per side)) panel stage\n")
        for (job, prec, b), v in sorted(table.items()):
            fh.write(f"{job} {prec} {b} {v}\n" if job in ("MV", "PANEL", "SHAPE") else f"{job} {prec} {b} {v[0]} {v[1]}\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="2,3,4,5")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.txt"))
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    t = tune([int(x) for x in a.configs.split(",")], log=lambda *x: print(*x, flush=True))
    write_table(t, a.out)
    print("wrote", a.out)

#!/usr/bin/env python3
"""Benchmark of the multilevel BDDC hot path on one MI355X.

Metric: time-to-solution at relative residual 1e-8 (set-up + solve), plus
BDDC preconditioner applications per second, mixed precision vs FP64.

A step is one pass of the whole path on the benchmark workload: host
planning, numeric set-up of every level (assembly, partial Cholesky of the
subdomain matrices, constrained local operators, coarse bases and matrices,
next-level assembly, top coarse factor), condensation, BDDC-PCG to
||r||/||g|| < 1e-8 and interior recovery.  Inputs are resident in device
memory before the timed region.

The default workload is the largest single-GPU configuration: 3D linear
elasticity on a 96^3 hexahedral mesh of the unit cube (2,709,792 DOFs),
12x12x12 = 1728 subdomains of 8^3 elements, corners + edge + face
averages, three levels (4x4x4 level-2 groups -> 27 level-2 subdomains,
top coarse problem of 294 DOFs), per-element E = 10^(3U), U ~ U(0,1)
(seed 0), nu = 0.3, body force (0, 0, -1), face x = 0 clamped.

Prints one JSON line: time-to-solution of the mixed mode as the value, both modes in detail, the
rooflines of the dominant kernels, and the oracle timed on a sample of the workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solution at rel. res 1e-8 + BDDC applies/s, mixed vs FP64"
PEAK = {"fp64": 78.6, "fp32": 157.3}       # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                           # GB/s


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_apply_bytes(s, precision: str) -> dict:
    """Bytes an apply must stream with explicit local operators (per level):
    the lower triangle of G_i, Psi_i twice (restriction and prolongation),
    and on levels >= 2 the interior operators K_II^{-1} (triangle) and
    K_II^{-1} K_IG (twice).  Plus the S^ triangle per PCG iteration (FP64)."""
    import numpy as np
    L = s.problem.n_levels
    esz = 4 if precision == "mixed" else 8
    total = 0.0
    schur = 0.0
    for lev in range(1, L):
        sz = s.subdomain_sizes(lev).astype(np.float64)
        nI, nG, nc = sz[:, 0], sz[:, 1], sz[:, 2]
        total += esz * float(np.sum(nG * (nG + 1) / 2 + 2 * nG * nc))
        if lev == 1:
            schur = 8.0 * float(np.sum(nG * (nG + 1) / 2))
        else:
            kes = esz
            total += kes * float(np.sum(nI * (nI + 1) / 2 + 2 * nI * nG))
    top = s.subdomain_sizes(L).astype(np.float64)
    total += 8.0 * float(np.sum(top[:, 0] * (top[:, 0] + 1) / 2))
    return {"apply": total, "schur": schur}


# Source sections whose PMC traffic figures are valid only for the code they were measured on.
KERNEL_SOURCES = {
    "k_tile_mm": ("dense.hip", "// Register staging of NE consecutive elements",
                  "// ----------------------------------------------------- preconditioner set-up"),
    "k_mv_tiles": ("apply.hip", "// ---------------------------------------------------------------- tile mv",
                   "// Sum of the partial tiles of one output tile"),
}


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    fname, a, b = KERNEL_SOURCES[kernel.split("<")[0]]
    src = open(os.path.join(ROOT, "paper_1201_5991_amd", "csrc", fname)).read()
    return hashlib.sha256(src[src.index(a):src.index(b)].encode()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, per_launch: float):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (profiles/pmc_traffic.json), or None when the summary was taken on
    another workload, another kernel source, or launches of another size
    (`per_launch`: the algorithmic flops or bytes of one launch)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("workload_name") != workload or k.get("source_hash") != kernel_source_hash(kernel):
        return None
    ref = k.get("algorithmic_per_launch")
    if not ref or abs(ref - per_launch) > 0.01 * per_launch:
        return None
    return k.get("hbm_bytes_per_launch")


MV_KERNEL = {("schur_mv", "mixed"): "k_mv_tiles<double, double>", ("schur_mv", "fp64"): "k_mv_tiles<double, double>",
             ("precond_mv", "mixed"): "k_mv_tiles<float, float>", ("precond_mv", "fp64"): "k_mv_tiles<double, double>"}


def rooflines(R: dict, mode: str, workload: str):
    """Roofline of the dominant kernel class of one step (largest device time
    per step: a set-up class once, a product class once per PCG iteration),
    and of the dominant set-up kernel."""
    prof = {k: v for k, v in R["profile"].items() if k != "jobs"}
    its = R["iterations"]
    per_step = {}
    for k, v in prof.items():
        if not v["launches"]:
            continue
        per_step[k] = v["time_s"] / v["launches"] * its if k.endswith("_mv") else v["time_s"]
    setup_cls = [k for k in per_step if not k.endswith("_mv")]

    def mfma(k):
        v = prof[k]
        prec = "fp32" if k.endswith("fp32") else "fp64"
        achieved = v["flops"] / v["time_s"] * 1e-12 if v["time_s"] > 0 else 0.0
        kern = f"k_tile_mm<{'float' if prec == 'fp32' else 'double'}, false>" if k.startswith("update") else k
        r = {"kernel": kern, "bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
             "frac": achieved / PEAK[prec], "traffic": None,
             "traffic_unit": "HBM bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
             "launches": v["launches"], "avg_launch_ms": v["time_s"] / max(v["launches"], 1) * 1e3,
             "flops_per_launch": v["flops"] / max(v["launches"], 1),
             # lower bound on a launch's HBM bytes: each updated 64x64 tile read and written once
             "c_tile_bytes_per_launch": v["tiles"] / max(v["launches"], 1) * 2 * 64 * 64 * (4 if prec == "fp32" else 8)}
        if k.startswith("update"):
            r["traffic"] = measured_traffic(kern, workload, r["flops_per_launch"])
        return r

    def hbm(k):
        v = prof[k]
        n = max(v["launches"], 1)
        avg = v["time_s"] / n
        per = v["bytes"] / n
        achieved = per / avg * 1e-9 if avg > 0 else 0.0
        kern = MV_KERNEL[(k, mode)]
        return {"kernel": kern, "product": "S^ = sum R_i^T S_i R_i (FP64)" if k == "schur_mv" else "level-1 G_i r_i",
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": measured_traffic(kern, workload, per),
                "traffic_unit": "HBM bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes_per_launch": per, "launches": v["launches"], "avg_launch_ms": avg * 1e3,
                "device_ms_per_step": avg * its * 1e3}

    dom = max(per_step, key=per_step.get)
    roof = hbm(dom) if dom.endswith("_mv") else mfma(dom)
    roof_setup = mfma(max(setup_cls, key=per_step.get)) if setup_cls else None
    return roof, roof_setup


def run_mode(prob, f, precision: str, steps: int, warmup: int, applies: int, panel: int = 0, graph: bool = True,
             lookahead: bool = False, fp32_form: int = 0):
    import torch
    from paper_1201_5991_amd import Solver
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    s = Solver(precision=precision, panel_tiles=panel, use_graph=graph, lookahead=lookahead, mfma_f32=fp32_form)
    mem = None
    t_cold = None
    for _ in range(warmup):
        tc = time.perf_counter()
        s.setup(prob)
        s.solve(f)
        torch.cuda.synchronize()
        if t_cold is None:
            t_cold = time.perf_counter() - tc
            mem = torch.cuda.memory_allocated() - m0   # the handle's device blocks (set-up + solve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        s.setup(prob)
        u, st = s.solve(f)
    torch.cuda.synchronize()
    tts = (time.perf_counter() - t0) / steps
    _log(f"[{precision}] tts {tts:.4f} s, its {st['iterations']}, rel_res {st['rel_res']:.2e}")
    # applies/s on a fixed seeded vector (the whole apply: restriction, local
    # solves, coarse levels, averaging), and the S^ product alone
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    r = torch.randn(s.n_iface, dtype=torch.float64, device="cuda", generator=gen)
    z = torch.empty_like(r)
    x = torch.empty_like(r)
    for _ in range(10):
        s.apply_into(r, z)
        s.apply_schur_into(r, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(applies):
        s.apply_into(r, z)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) * 1e-3 / applies
    e0.record()
    for _ in range(applies):
        s.apply_schur_into(r, x)
    e1.record()
    torch.cuda.synchronize()
    t_schur = e0.elapsed_time(e1) * 1e-3 / applies
    nbytes = algorithmic_apply_bytes(s, precision)
    # profiled pass: HIP events inside the library around every factorization
    # launch of one set-up and around the S^ / G tile-product kernels of
    # eager applies, each on the stream the launch runs on
    s.set_profiling(True)
    s.setup(prob)
    for _ in range(applies):
        s.apply_schur_into(r, x)
        s.apply_into(r, z)
    torch.cuda.synchronize()
    prof = s.profile()
    s.set_profiling(False)
    res = {
        "tts_s": tts,
        "tts_first_call_s": t_cold,
        "t_plan_s": st["t_plan"],
        "t_setup_num_s": st["t_setup_num"],
        "t_solve_s": st["t_solve"],
        "iterations": st["iterations"],
        "rel_res": st["rel_res"],
        "lambda_min": st["lambda_min"],
        "lambda_max": st["lambda_max"],
        "applies_per_s": 1.0 / t_apply,
        "apply_ms": t_apply * 1e3,
        "apply_alg_GBps": nbytes["apply"] / t_apply * 1e-9,
        "schur_ms": t_schur * 1e3,
        "schur_alg_GBps": nbytes["schur"] / t_schur * 1e-9,
        "device_memory_GB": None if mem is None else mem * 1e-9,
        "profile": prof,
    }
    s.destroy()
    return res


def _oracle_record(workload: str):
    """The committed full-size oracle run of `workload` (written by
    tests/golden/make_golden.py, which calls only the oracle), or None."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "*.json"))):
        try:
            d = json.load(open(path))
        except (OSError, ValueError):
            continue
        if d.get("workload") == workload and "oracle_time_s" in d and isinstance(d["oracle_time_s"], dict):
            return {"file": os.path.relpath(path, ROOT), "time_s": d["oracle_time_s"], "iterations": d["pcg"]["iterations"],
                    "host": d.get("host")}
    return None


def cpu_baseline(w, levels: int, gpu_iterations: int):
    """The FP64 oracle, as it stands, on a bounded sample of the benchmark
    workload, scaled to the whole workload's time-to-solution.

    Sample: the corner block of 5x5x5 of the workload's subdomains (the same
    subdomain size and the same element moduli, the clamped face included),
    run through the oracle's full pipeline (set-up, condensation, PCG to
    1e-8, recovery) at two levels.  The oracle's work is a loop over
    subdomains, so its set-up, condensation and recovery scale with the
    subdomain count, and its PCG with the subdomain count times the
    iteration count; the full workload's iteration count is the oracle's own
    when its full-size run is committed, else the GPU's."""
    import numpy as np
    from oracle import fem
    from oracle.bddc import MultilevelBDDC
    from oracle.krylov import pcg
    from workloads import box_workload
    from workloads.gen import uniform_cuts
    try:
        from threadpoolctl import threadpool_info
        import numpy  # noqa: F401  (BLAS loaded before the query)
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    nsub_axis = [len(c) - 1 for c in w.cuts]
    el = [int(np.diff(c)[0]) for c in w.cuts]
    k = 5
    n = [k * e for e in el]
    young = w.young.reshape(w.n_el[::-1])[: n[2], : n[1], : n[0]].ravel()
    ws = box_workload("sample", "elasticity", tuple(n), [uniform_cuts(n[d], k) for d in range(3)], young=young)
    nsub_full = int(np.prod(nsub_axis))
    scale = nsub_full / k ** 3
    t0 = time.perf_counter()
    b = MultilevelBDDC(ws, n_levels=2)
    t_setup = time.perf_counter() - t0
    _, fs = fem.assemble_global(ws)
    t1 = time.perf_counter()
    g = b.condense(fs)
    t_cond = time.perf_counter() - t1
    t2 = time.perf_counter()
    res = pcg(b.schur_apply, g, b.apply, tol=1e-8)
    t_pcg = time.perf_counter() - t2
    t3 = time.perf_counter()
    b.recover(fs, res.x)
    t_rec = time.perf_counter() - t3
    rec = _oracle_record(w.name)
    its_full = rec["iterations"] if rec else gpu_iterations
    per_it = t_pcg / max(res.iterations, 1)
    value = scale * (t_setup + t_cond + t_rec + per_it * its_full)
    out = {"value": value, "unit": "s (time-to-solution of the whole workload, scaled from the sample)",
           "cores": int(cores), "kind": "oracle",
           "sample": (f"FP64 oracle (SciPy SuperLU per subdomain, NumPy) on the corner {k}x{k}x{k} block of the workload's "
                      f"subdomains ({n[0]}x{n[1]}x{n[2]} elements, the same 8^3-element subdomains and moduli), 2 levels: "
                      f"set-up {t_setup:.2f} s, condensation {t_cond:.2f} s, {res.iterations} PCG iterations "
                      f"{t_pcg:.2f} s, recovery {t_rec:.2f} s; scaled x{scale:g} subdomains and to {its_full} "
                      f"iterations ({'the oracle' if rec else 'the GPU'}'s count on the full workload)"),
           "sample_s": t_setup + t_cond + t_pcg + t_rec}
    if rec:
        out["full_run"] = {"note": "the oracle's measured run on the whole workload, committed with the parity fixtures",
                           **rec}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--applies", type=int, default=100)
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--panel", type=int, default=0, help="tile columns per factorization panel (0 = library default)")
    ap.add_argument("--no-graph", action="store_true", help="launch PCG iterations eagerly instead of replaying a HIP graph")
    ap.add_argument("--fp32-form", type=int, default=0, choices=(0, 16, 32, 3),
                    help="form of the FP32 tile products: 16 / 32 (FP32 MFMA shape), 3 (split bf16); 0 = tune table")
    ap.add_argument("--lookahead", action="store_true",
                    help="factor on two streams (next panel beside the bulk trailing update)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 512 MiB (3 times) to calibrate PMC byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for {args.gpus}); a multi-GPU run would give each GPU "
              f"a block of level-2 groups and exchange interface sums between neighbours, which is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1201_5991_amd import Problem
    from workloads import config

    w = config(args.config, levels=args.levels) if args.config in (2, 3) else config(args.config)
    prob = Problem(w)
    f = torch.tensor(prob.load_vector(), device="cuda")
    torch.cuda.synchronize()
    counts = prob.counts()
    modes = args.modes.split(",")
    out = {}
    for m in modes:
        out[m] = run_mode(prob, f, m, args.steps, args.warmup, args.applies, args.panel, not args.no_graph,
                          args.lookahead, args.fp32_form)
    main_mode = "mixed" if "mixed" in out else modes[0]
    R = out[main_mode]
    roof, roof_setup = rooflines(R, main_mode, w.name)
    line = {
        "metric": METRIC,
        "value": R["tts_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["tts_s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_mode == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dofs": int(prob.n_dofs), "levels": int(prob.n_levels),
                   "subdomains": [int(c[0]) for c in counts], "interface": int(counts[0][1]),
                   "coarse": [int(c[2]) for c in counts], "value_mode": main_mode,
                   "pcg_graph": not args.no_graph, "lookahead": args.lookahead,
                   **({"fp32_form": args.fp32_form} if args.fp32_form else {})},
        "applies_per_s": R["applies_per_s"],
        "roofline": roof,
        "roofline_setup": roof_setup,
    }
    for m in modes:
        d = dict(out[m])
        jobs = d["profile"].get("jobs", {})
        d["profile"] = {k: {"time_ms": v["time_s"] * 1e3, "tflops": (v["flops"] / v["time_s"] * 1e-12 if v["time_s"] else 0.0),
                            "GBps": (v["bytes"] / v["time_s"] * 1e-9 if v["time_s"] else 0.0),
                            "launches": v["launches"]} for k, v in d["profile"].items() if k != "jobs"}
        d["profile"]["jobs"] = jobs
        line[m] = d
    if "fp64" in out and "mixed" in out:
        line["mixed_speedup"] = {"tts": out["fp64"]["tts_s"] / out["mixed"]["tts_s"],
                                 "apply": out["mixed"]["applies_per_s"] / out["fp64"]["applies_per_s"]}
    line["apply_roofline"] = {"bound": "hbm", "achieved": R["apply_alg_GBps"], "peak": HBM_PEAK, "unit": "GB/s",
                              "frac": R["apply_alg_GBps"] / HBM_PEAK}
    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 2 * a.numel() * 8
    if not args.no_cpu_baseline:
        _log("[cpu baseline] oracle sample ...")
        line["cpu_baseline"] = cpu_baseline(w, int(prob.n_levels), int(out[main_mode]["iterations"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

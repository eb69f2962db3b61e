"""Benchmark: long-range PSWF fast Ewald (potentials + forces + energy) on one MI355X.

Workload: water-like box of 10,000 rigid 3-site molecules (n = 30,000 charges, L = 6.688 nm,
1 g/cm^3, SPC/E-like charges), eps = 1e-6 absolute RMS with the parameters of Alg. 3 on a 64^3
grid (P = 13). One step = one full pass of the pipeline (binning, spreading, FFT with fused
scaling, inverse FFT, interpolation of phi and forces, self term and energy) on inputs resident
in HBM. The headline value is the float32 path; the float64 path is timed on the same system,
and a batch of 256 independent systems is timed batched (one HIP graph) and sequentially.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
                       [--no-comparison]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "long-range particles/s (φ+forces) at ε=1e-6 FP32 vs FP64; % HBM roofline"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6    # float64 vector FMA (256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz); the float64 MFMA peak is the same
STAGES = ["bin", "spread", "fft_x", "fft_y", "fft_z_scale", "ifft_y", "ifft_x", "gather"]


def stage_work(stage: str, n: int, m: int, P: int, deg: int, elem: int):
    """Algorithmic work of one launch of a stage: ("mfma" or "alu", flops) or ("hbm", bytes).

    spread: per particle 3P Horner chains (2 deg flops), P^2 products q w_z w_y (2 flops),
            P^3 multiply-adds into the grid (2 flops); the multiply-adds run as a float64
            matrix product on the matrix cores.
    gather: per particle 6P Horner chains for values and derivatives (2 deg flops each),
            P^3 points x 2 multiply-adds (phi and d/dx sums), P^2 lines x 3, P planes x 4.
    FFT passes: one read and one write of the grid or the half spectrum.
    bin: read positions and charges, write the sorted record, cell, permutation.
    """
    half = m * m * (m // 2 + 1) * 2 * elem
    real = m ** 3 * elem
    if stage == "spread":
        return "mfma", n * (3 * P * 2 * deg + 2 * P * P + 2 * P ** 3)
    if stage == "gather":
        return "alu", n * (6 * P * 2 * deg + 4 * P ** 3 + 6 * P * P + 8 * P)
    if stage == "fft_x":
        return "hbm", real + half
    if stage == "ifft_x":
        return "hbm", half + real
    if stage in ("fft_y", "fft_z_scale", "ifft_y"):
        return "hbm", 2 * half
    if stage == "bin":
        return "hbm", n * (4 * elem + 4 * elem + 4 + 4 + 4)
    raise KeyError(stage)


STAGE_KERNEL = {"spread": ("k_spread", "k_spread_cols", "k_spread_mfma"), "gather": ("k_gather",), "fft_x": ("k_fft_x_r2c",),
                "fft_y": ("k_fft_cols",), "fft_z_scale": ("k_fft_cols",), "ifft_y": ("k_fft_cols",),
                "ifft_x": ("k_fft_x_c2r",), "bin": ("k_bin_count",)}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_water_box_n30000.md")
TRAFFIC_FILE_N1E6 = os.path.join(ROOT, "profiles", "traffic_uniform_n1e6.md")
# the device code whose counters the traffic file holds; any change to the code voids them
KERNEL_SOURCES = ("kernels.hip", "kernels.hpp", "particles.hip", "device_common.hpp")


def code_only(text: str) -> str:
    """C++ source with comments removed and every run of blank space made one space (string
    and character literals kept), so that editing a comment leaves the hash unchanged."""
    import re
    token = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/', re.S)
    stripped = token.sub(lambda m: " " if m.group(0).startswith("/") else m.group(0), text)
    return " ".join(stripped.split())


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_16591_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


LDS_FILE = os.path.join(ROOT, "profiles", "lds_water_box_n30000.md")


def _profile_blob(path, workload: str = "water_box_n30000"):
    """The machine-readable block of a committed counter summary, or None when it is missing,
    was taken on other kernel code or on another workload."""
    try:
        with open(path) as f:
            text = f.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("workload", "water_box_n30000") != workload:
        return None
    return blob if blob.get("kernel_source_sha256") == kernel_source_sha256() else None


def _stage_kernels(blob_keys, stage: str, prec_ctype: str):
    prefixes = tuple(f"{name}<{prec_ctype}" for name in STAGE_KERNEL[stage])
    hits = [k for k in blob_keys if k.startswith(prefixes)]
    if stage == "bin":   # the counting sort is three launches: count, scan, scatter
        hits += [k for k in blob_keys if k == "k_scan" or k.startswith(f"k_bin_scatter<{prec_ctype}")]
    return hits


def measured_traffic(stage: str, prec_ctype: str, workload: str = "water_box_n30000"):
    """HBM bytes per launch of the stage's kernel(s) from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, calibrated against a plain copy), or None when the summary
    is missing or was taken on other kernel sources."""
    blob = _profile_blob(TRAFFIC_FILE_N1E6 if workload == "uniform_n1e6" else TRAFFIC_FILE, workload)
    if blob is None:
        return None
    per = blob.get("bytes_per_launch", {})
    hits = _stage_kernels(per.keys(), stage, prec_ctype)
    if not hits or (stage != "bin" and len(hits) != 1):
        return None
    return sum(per[k] for k in hits)


def measured_lds(stage: str, prec_ctype: str, workload: str = "water_box_n30000"):
    """LDS instructions and LDS bank-conflict cycles per launch of the stage's kernel(s) from the
    committed counter summary, or None."""
    blob = _profile_blob(LDS_FILE, workload)
    if blob is None:
        return None
    per = blob.get("per_launch", {})
    hits = _stage_kernels(per.keys(), stage, prec_ctype)
    if not hits or (stage != "bin" and len(hits) != 1):
        return None
    return {c: sum(per[k][c] for k in hits) for c in ("lds_instr", "lds_bank_conflict_cycles", "valu_instr")}


def kernel_rooflines(stage_ms: dict, n: int, m: int, P: int, deg: int, elem: int, prec_ctype: str,
                     workload: str = "water_box_n30000"):
    """Per stage: event-timed duration, the algorithmic work and its roofline fraction, the HBM
    traffic the counters measured (GB/s against 8 TB/s) and the LDS bank-conflict share of the
    compute units' cycles (2.4 GHz x 256 CUs)."""
    out = {}
    for st in STAGES:
        us = stage_ms[st] * 1e3
        kind, work = stage_work(st, n, m, P, deg, elem)
        row = {"us": us}
        if kind in ("alu", "mfma"):
            peak = PEAK_FP64_TFLOPS
            row.update({"bound": kind, "flops": work, "tflops": work / us * 1e-6, "frac_fp64_peak": work / us * 1e-6 / peak})
        else:
            row.update({"bound": "hbm", "algorithmic_bytes": work, "gbs": work / us * 1e-3,
                        "frac_hbm_peak": work / us * 1e-3 / PEAK_HBM_GBS})
        t = measured_traffic(st, prec_ctype, workload)
        if t is not None:
            row.update({"measured_bytes": t, "measured_gbs": t / us * 1e-3, "measured_frac_hbm_peak": t / us * 1e-3 / PEAK_HBM_GBS})
        lds = measured_lds(st, prec_ctype, workload)
        if lds is not None:
            row.update({"lds_instr": lds["lds_instr"],
                        "lds_conflict_share": lds["lds_bank_conflict_cycles"] / (us * 2400.0 * 256)})
        out[st] = row
    return out


def cpu_baseline(x, q, L, eps, m, tol_mode="abs", sample=None, label="full water box"):
    """The float64 oracle of the same computation (Alg. 2 in NumPy, oracle/fast.py), single-
    threaded, timed on this host: on the full system, or on its first `sample` particles with
    the full system's parameters (grid and window), when the whole would take minutes."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fast, params
    if tol_mode == "abs":
        p = params.choose(eps, L, m=m, q_l2=float(np.linalg.norm(q)), tol_mode="abs")
    else:
        p = params.choose(eps, L, m=m)
    xs, qs = (x, q) if sample is None else (x[:sample], q[:sample])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        fast.fast_longrange(xs, qs, p, grad=True)
        dt = time.perf_counter() - t0
    what = f"{label} (n={len(qs)})" if sample is None else f"first {len(qs)} of the n={len(q)} {label} particles, same m and P"
    return {"value": len(qs) / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}, one evaluation of oracle/fast.py (Alg. 2, float64 NumPy, phi and gradients) "
                      f"taking {dt:.2f} s on 1 thread"}


def bench_ensemble(steps: int, warmup: int):
    """Batched vs sequential: 256 independent neutral systems (n log-uniform in [500, 20000],
    L uniform in [0.5, 2], uniform positions, +-1 charges), each with its own eps = 1e-6
    parameters (Alg. 3, relative mode, 64-neighbour cutoff rule), float32, phi + forces +
    energies. Batched: one plan over all systems, tiles from the autotuner, replayed as one HIP
    graph (and, for reference, called eagerly). Sequential: one default plan per system, called
    one after another."""
    import numpy as np
    import torch
    import paper_2602_16591_amd as pw
    import workloads as W
    from paper_2602_16591_amd.autotune import autotune_batch

    dev = torch.device("cuda:0")
    ens = W.ensemble()
    params = [pw.choose_params(1e-6, L, n=len(q)) for _, q, L in ens]
    counts = [len(q) for _, q, _ in ens]
    n_total = sum(counts)
    X = torch.as_tensor(np.concatenate([x for x, _, _ in ens]), dtype=torch.float32, device=dev)
    Q = torch.as_tensor(np.concatenate([q for _, q, _ in ens]), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    plan, tiles, report = autotune_batch(params, counts, X, Q, "fp32", targets=(None, 64, 256), reps=5)
    tune_s = time.perf_counter() - t0
    runner = plan.graph(X, Q)

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / k

    g_s = timed(runner, steps)
    phi = torch.empty(n_total, dtype=torch.float32, device=dev)
    F = torch.empty((n_total, 3), dtype=torch.float32, device=dev)
    E = torch.empty(len(ens), dtype=torch.float64, device=dev)
    e_s = timed(lambda: plan.compute(X, Q, phi=phi, force=F, energy=E), steps)
    stage_ms = {}
    for st in STAGES:
        plan.timing_enable(st, 8)
        for _ in range(4):
            plan.compute(X, Q, phi=phi, force=F, energy=E)
        ms, calls = plan.timing_read()
        stage_ms[st] = ms / max(calls, 1)
    plan.timing_enable(None)
    singles = [pw.Plan(p, "fp32", n_max=c) for p, c in zip(params, counts)]
    views = [(X[o:o + c], Q[o:o + c], phi[o:o + c], F[o:o + c], E[k:k + 1])
             for k, (o, c) in enumerate(zip(plan.offsets, plan.counts))]

    def sequential():
        for sp, (x, q, ph, f, e) in zip(singles, views):
            sp.compute(x, q, phi=ph, force=f, energy=e)

    s_s = timed(sequential, max(2, steps // 4))
    for sp in singles:
        sp.close()
    P_counts = {}
    for p in params:
        P_counts[p.P] = P_counts.get(p.P, 0) + 1
    return {
        "workload": "ensemble_256_systems", "n_total": n_total, "systems": len(ens),
        "m_range": [min(p.m for p in params), max(p.m for p in params)], "P_counts": P_counts,
        "batched_graph": {"value": n_total / g_s, "unit": "particles/s", "ms_per_step": g_s * 1e3},
        "batched_eager": {"value": n_total / e_s, "unit": "particles/s", "ms_per_step": e_s * 1e3},
        "sequential": {"value": n_total / s_s, "unit": "particles/s", "ms_per_step": s_s * 1e3,
                       "plans": len(singles)},
        "speedup_graph_vs_sequential": s_s / g_s,
        "autotune": {"seconds": tune_s,
                     "candidates": [{"target": "tile 8" if t is None else t, "ms": ms} for t, _, ms in report],
                     "tiles_hist": {str(b): tiles.count(b) for b in sorted(set(tiles))}},
        "stage_us_batched": {k: v * 1e3 for k, v in stage_ms.items()},
    }


# Comparison configurations at the paper's resolutions (split, window, eps, m from the table, P):
# Table 3 at eps = 1e-6 (PSWF/PSWF, Gaussian/PSWF, Gaussian/Gaussian) and Table 4 at eps = 1e-5
# (B-spline windows of order 4, 6, 8 with the PSWF and the Gaussian split; PSWF/PSWF from Table 3).
COMPARISON = [
    ("PP", "pswf", "pswf", 1e-6, 42, 10), ("GP", "gauss", "pswf", 1e-6, 79, 10),
    ("GG", "gauss", "gauss", 1e-6, 80, 15),
    ("PP", "pswf", "pswf", 1e-5, 35, 9),
    ("PB4", "pswf", "bspline", 1e-5, 154, 4), ("PB6", "pswf", "bspline", 1e-5, 66, 6),
    ("PB8", "pswf", "bspline", 1e-5, 49, 8),
    ("GB4", "gauss", "bspline", 1e-5, 230, 4), ("GB6", "gauss", "bspline", 1e-5, 101, 6),
    ("GB8", "gauss", "bspline", 1e-5, 78, 8),
]


def bench_comparison(steps: int, warmup: int, n: int = 100_000):
    """MI355X time of the paper's split/window configurations at equal accuracy: the grid sizes
    and supports of Tables 3 and 4 (m rounded up to an FFT size), n uniform particles with
    N(0,1) charges shifted to neutrality in the unit box, r_c = 0.1 (the tables' setup, with
    more particles), float32, phi + forces + energy, one graph replay per step."""
    import numpy as np
    import torch
    import paper_2602_16591_amd as pw
    import workloads as W

    dev = torch.device("cuda:0")
    x, q, L = W.paper_default(n, seed=W.SEED_BASE + 7)
    X = torch.as_tensor(x, dtype=torch.float32, device=dev)
    Q = torch.as_tensor(q, dtype=torch.float32, device=dev)
    rows = []
    for name, split, window, eps, m_tab, P in COMPARISON:
        m = m_tab
        while True:   # next even size with prime factors 2, 3, 5, 7
            r = m
            for f in (2, 3, 5, 7):
                while r % f == 0:
                    r //= f
            if r == 1 and m % 2 == 0:
                break
            m += 1
        c = pw.variant_params(split, window, L, 0.1, math.log(1.0 / eps), m, P, eps=eps)
        plan = pw.Plan(c, "fp32", n_max=n)
        runner = plan.graph(X, Q)
        for _ in range(warmup):
            runner()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            runner()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / steps * 1e3
        rows.append({"config": name, "split": split, "window": window, "eps": eps, "m_table": m_tab, "m": m,
                     "P": P, "ms_per_step": ms})
        del runner
        plan.close()
    ref = {eps: next(r["ms_per_step"] for r in rows if r["config"] == "PP" and r["eps"] == eps) for eps in (1e-6, 1e-5)}
    for r in rows:
        r["time_vs_PP"] = r["ms_per_step"] / ref[r["eps"]]
    # oversampled grids: Alg. 3 parameters (eps = 1e-6, r_c = 0.1) on grids sigma times finer with
    # the smaller support they allow
    over = []
    base = pw.choose_params(1e-6, L, rc=0.1)
    for sigma in (1.0, 1.5, 2.0):
        c = pw.oversample_params(base, sigma)
        plan = pw.Plan(c, "fp32", n_max=n)
        runner = plan.graph(X, Q)
        for _ in range(warmup):
            runner()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            runner()
        torch.cuda.synchronize()
        over.append({"sigma": sigma, "m": c.m, "P": c.P, "cw": c.cw,
                     "ms_per_step": (time.perf_counter() - t) / steps * 1e3})
        del runner
        plan.close()
    return {"workload": f"uniform_n{n}_unit_box_rc0.1", "prec": "fp32", "rows": rows, "oversampled_eps1e-6": over}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("water_box_n30000", "uniform_n1e6"), default="water_box_n30000",
                    help="water box (default, the headline) or n = 1e6 uniform (float32 at eps 1e-6 on 128^3, "
                         "float64 at eps 1e-10 with the same r_c)")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential ensemble")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the split/window comparison at the paper's resolutions")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the measurement, copy a device buffer of this many MiB three times (a kernel of "
                         "known traffic, to calibrate profiler byte counters); not part of the result")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the pipeline runs on a single MI355X; "
              "multi-GPU sharding is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2602_16591_amd as pw
    import workloads as W

    dev = torch.device("cuda:0")
    water = args.workload == "water_box_n30000"
    if water:
        x, q, L = W.config("water_n30000")
        eps, m = 1e-6, 64
        params = pw.choose_params(eps, L, m=m, q_l2=float(np.linalg.norm(q)), tol_mode="abs")
        params_of = {"fp32": params, "fp64": params}
    else:
        x, q, L = W.config("uniform_n1e6")
        eps, m = 1e-6, 128
        params = pw.choose_params(eps, L, m=m)
        params_of = {"fp32": params, "fp64": pw.choose_params(1e-10, L, rc=params.rc)}
    n = len(q)
    # both precisions see the same float32-representable inputs, so the float32/float64
    # comparison below isolates arithmetic error from input quantisation
    x = x.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    P = params.P
    results = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        plan = pw.Plan(params_of[prec], prec, n_max=n)
        X = torch.as_tensor(x, dtype=dt, device=dev).contiguous()
        Q = torch.as_tensor(q, dtype=dt, device=dev).contiguous()
        phi = torch.empty(n, dtype=dt, device=dev)
        F = torch.empty((n, 3), dtype=dt, device=dev)
        E = torch.empty(1, dtype=torch.float64, device=dev)

        def step():
            plan.compute(X, Q, phi=phi, force=F, energy=E)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # untimed calibration: average duration of every stage, to pick the dominant kernel
        stage_ms = {}
        for st in STAGES:
            plan.timing_enable(st, 16)
            for _ in range(8):
                step()
            ms, calls = plan.timing_read()
            stage_ms[st] = ms / max(calls, 1)
        plan.timing_enable(None)
        dom = max(stage_ms, key=stage_ms.get)
        plan.timing_enable(dom, args.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        dom_ms_total, dom_calls = plan.timing_read()
        plan.timing_enable(None)
        results[prec] = dict(elapsed=elapsed, dom=dom, dom_ms=dom_ms_total / max(dom_calls, 1), stage_ms=stage_ms,
                             phi=phi.double().cpu().numpy(), F=F.double().cpu().numpy(), E=float(E.cpu()[0]),
                             deg=pw.host_tables(params_of[prec], prec)["deg"], elem=4 if prec == "fp32" else 8)
        if not water:
            plan.close()
            continue
        # the full Ewald sum (real-space residual added), same inputs, outside the headline
        def step_total():
            plan.compute(X, Q, phi=phi, force=F, energy=E, total=True)

        for _ in range(5):
            step_total()
        plan.timing_enable("local", 16)
        for _ in range(8):
            step_total()
        lms, lcalls = plan.timing_read()
        plan.timing_enable(None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ksteps = max(10, args.steps // 4)
        for _ in range(ksteps):
            step_total()
        torch.cuda.synchronize()
        total_s = (time.perf_counter() - t1) / ksteps
        results[prec + "_total"] = {"value": n / total_s, "unit": "particles/s", "ms_per_step": total_s * 1e3,
                                    "local_overlapped_us": lms / max(lcalls, 1) * 1e3}
        plan.close()

    r = results["fp32"]
    value = n * args.steps / r["elapsed"]
    kind, work = stage_work(r["dom"], n, m, P, r["deg"], r["elem"])
    secs = r["dom_ms"] * 1e-3
    if kind in ("alu", "mfma"):
        # the particle kernels compute window values, products and sums in float64 in both
        # precisions; the spread's sums run on the matrix cores, whose float64 peak on MI355X
        # equals the float64 vector rate
        achieved = work / secs / 1e12
        roof = {"bound": kind, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
    else:
        achieved = work / secs / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof["traffic"] = measured_traffic(r["dom"], "float", args.workload)
    roof.update({"kernel": r["dom"], "avg_launch_us": r["dom_ms"] * 1e3, "work_per_launch": work})
    r64 = results["fp64"]
    p64 = params_of["fp64"]
    if water:
        config = {"workload": "water_box_n30000", "n": n, "L_nm": L, "eps": eps, "tol_mode": "abs", "m": m, "P": P,
                  "rc_nm": params.rc, "parallelism": "single GPU"}
    else:
        config = {"workload": "uniform_n1e6", "n": n, "L": L, "eps": eps, "tol_mode": "rel", "m": m, "P": P,
                  "rc": params.rc, "fp64": {"eps": 1e-10, "m": p64.m, "P": p64.P}, "parallelism": "single GPU"}
    out = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["elapsed"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": config,
        "roofline": roof,
        "stage_us_fp32": {k: v * 1e3 for k, v in r["stage_ms"].items()},
        "fp64": {"value": n * args.steps / r64["elapsed"], "unit": "particles/s",
                 "ms_per_step": r64["elapsed"] / args.steps * 1e3,
                 "stage_us": {k: v * 1e3 for k, v in r64["stage_ms"].items()}},
        "kernels_fp32": kernel_rooflines(r["stage_ms"], n, m, P, r["deg"], r["elem"], "float", args.workload),
        "kernels_fp64": kernel_rooflines(r64["stage_ms"], n, p64.m, p64.P, r64["deg"], r64["elem"], "double",
                                         args.workload),
    }
    if water:
        phi_diff = float(np.linalg.norm(r["phi"] - r64["phi"]) / np.linalg.norm(r64["phi"]))
        phi_abs = float(np.sqrt(np.mean((r["phi"] - r64["phi"]) ** 2)))
        F_diff = float(np.linalg.norm(r["F"] - r64["F"]) / np.linalg.norm(r64["F"]))
        out["fp32_vs_fp64"] = {"phi_rel_l2": phi_diff, "phi_abs_rms": phi_abs, "force_rel_l2": F_diff,
                               "energy_rel": abs(r["E"] - r64["E"]) / abs(r64["E"])}
        out["total_ewald"] = {"note": "phi_far + phi_local + phi_self (real-space residual on the GPU), same workload; "
                                      "local_overlapped_us: the residual's span on its own stream, which it shares "
                                      "with the long-range kernels running at the same time",
                              "fp32": results["fp32_total"], "fp64": results["fp64_total"]}
    if not args.no_batched:
        out["batched"] = bench_ensemble(max(5, min(args.steps, 50)), max(2, min(args.warmup, 5)))
    if not args.no_comparison:
        out["comparison"] = bench_comparison(max(5, min(args.steps, 30)), max(2, min(args.warmup, 5)))
    if not args.no_cpu_baseline:
        if water:
            out["cpu_baseline"] = cpu_baseline(x, q, L, eps, m)
        else:
            out["cpu_baseline"] = cpu_baseline(x, q, L, eps, m, tol_mode="rel", sample=200_000,
                                               label="uniform")
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4, "launches": 3}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

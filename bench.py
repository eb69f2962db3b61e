"""Benchmark: long-range PSWF fast Ewald (potentials + forces + energy) on one MI355X.

Headline workload: water-like box of 10,000 rigid 3-site molecules (n = 30,000 charges,
L = 6.688 nm, 1 g/cm^3, SPC/E-like charges), eps = 1e-6 absolute RMS with the parameters of
Alg. 3 on a 64^3 grid (P = 13). One step = one full pass of the pipeline (binning, spreading,
FFT with fused scaling, inverse FFT, interpolation of phi and forces, self term and energy) on
inputs resident in HBM. The headline value is the float32 path; the float64 path is timed on the
same system. Alongside: the n = 1e6 uniform system (float32 at eps = 1e-6 on 128^3, float64 at
eps = 1e-10 on 216^3), a batch of 256 independent systems timed batched (one HIP graph) and
sequentially, the paper's split/window comparison configurations, and the float64 oracle on the
host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
                       [--no-comparison] [--no-large] [--workload water_box_n30000|uniform_n1e6]
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
PEAK_FP32_TFLOPS = 157.3   # float32 vector FMA (256 CU x 4 SIMD x 64 lanes x 2 flops x 2.4 GHz) and dense float32 MFMA
# plan precisions timed: float32 storage with float32 arithmetic in spreading and interpolation
# (the headline float32 path), float32 storage with float64 arithmetic, float64
PRECISIONS = ("fp32_arith", "fp32", "fp64")


def peak_tflops(prec: str) -> float:
    """Peak of the arithmetic the particle kernels of a plan precision run in."""
    return PEAK_FP32_TFLOPS if prec == "fp32_arith" else PEAK_FP64_TFLOPS
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


STAGE_KERNEL = {"spread": ("k_spread", "k_spread_cols", "k_spread_mfma"), "gather": ("k_gather", "k_gather_stream"), "fft_x": ("k_fft_x_r2c",),
                "fft_y": ("k_fft_cols",), "fft_z_scale": ("k_fft_cols", "k_fft_yz"), "ifft_y": ("k_fft_cols",),
                "ifft_x": ("k_fft_x_c2r",),
                # one-level sort (count, scan, scatter) or two-level sort (count, coarse, fine)
                "bin": ("k_bin_count1", "k_bin_scatter1", "k_bin_count", "k_bin_coarse", "k_bin_fine")}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_water_box_n30000.md")
TRAFFIC_FILE_N1E6 = os.path.join(ROOT, "profiles", "traffic_uniform_n1e6.md")
# the device code whose counters a summary holds, and its hash (comments and blank space aside)
from paper_2602_16591_amd.profile_summary import KERNEL_SOURCES, code_only, kernel_source_sha256  # noqa: E402,F401

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


# kernels with a template argument for the type of their window arithmetic, and its position:
# k_spread_mfma<T, P, D, B, A, column form>, k_gather<T, P, D, G>
ARITH_ARG = {"k_spread_mfma": 4, "k_gather": 3, "k_gather_stream": 3}


def _stage_kernels(blob_keys, stage: str, prec: str):
    """Names of the kernels that run a stage at a plan precision ("fp32_arith", "fp32", "fp64")."""
    ctype = "double" if prec == "fp64" else "float"
    arith = "float" if prec == "fp32_arith" else "double"
    hits = []
    for k in blob_keys:
        name = k.split("<", 1)[0]
        if name in STAGE_KERNEL[stage] and k.startswith(f"{name}<{ctype}"):
            args = k[len(name) + 1:-1].split(", ")
            if name not in ARITH_ARG or (len(args) > ARITH_ARG[name] and args[ARITH_ARG[name]] == arith):
                hits.append(k)
    if stage == "bin" and any(k.startswith("k_bin_count1<") for k in hits):   # the one-level sort's scan
        hits += [k for k in blob_keys if k == "k_scan"]
    return hits


def measured_traffic(stage: str, prec: str, workload: str = "water_box_n30000"):
    """HBM bytes per launch of the stage's kernel(s) from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, calibrated against a plain copy), or None when the summary
    is missing or was taken on other kernel sources."""
    blob = _profile_blob(TRAFFIC_FILE_N1E6 if workload == "uniform_n1e6" else TRAFFIC_FILE, workload)
    if blob is None:
        return None
    per = blob.get("bytes_per_launch", {})
    hits = _stage_kernels(per.keys(), stage, prec)
    if not hits or (stage != "bin" and len(hits) != 1):
        return None
    return sum(per[k] for k in hits)


def measured_lds(stage: str, prec: str, workload: str = "water_box_n30000"):
    """LDS instructions and LDS bank-conflict cycles per launch of the stage's kernel(s) from the
    committed counter summary, or None."""
    blob = _profile_blob(LDS_FILE, workload)
    if blob is None:
        return None
    per = blob.get("per_launch", {})
    hits = _stage_kernels(per.keys(), stage, prec)
    if not hits or (stage != "bin" and len(hits) != 1):
        return None
    return {c: sum(per[k][c] for k in hits) for c in ("lds_instr", "lds_bank_conflict_cycles", "valu_instr")}


def kernel_rooflines(stage_ms: dict, n: int, m: int, P: int, deg: int, elem: int, prec: str,
                     workload: str = "water_box_n30000"):
    """Per stage: event-timed duration, the algorithmic work and its roofline fraction (against the
    peak of the arithmetic the kernel runs in), the HBM traffic the counters measured (GB/s
    against 8 TB/s) and the LDS bank-conflict share of the compute units' cycles (2.4 GHz x 256
    CUs)."""
    out = {}
    for st in STAGES:
        us = stage_ms[st] * 1e3
        kind, work = stage_work(st, n, m, P, deg, elem)
        row = {"us": us}
        if kind in ("alu", "mfma"):
            peak = peak_tflops(prec)
            row.update({"bound": kind, "flops": work, "tflops": work / us * 1e-6, "peak_tflops": peak,
                        "frac_peak": work / us * 1e-6 / peak})
        else:
            row.update({"bound": "hbm", "algorithmic_bytes": work, "gbs": work / us * 1e-3,
                        "frac_hbm_peak": work / us * 1e-3 / PEAK_HBM_GBS})
        t = measured_traffic(st, prec, workload)
        if t is not None:
            row.update({"measured_bytes": t, "measured_gbs": t / us * 1e-3, "measured_frac_hbm_peak": t / us * 1e-3 / PEAK_HBM_GBS})
        lds = measured_lds(st, prec, workload)
        if lds is not None:
            row.update({"lds_instr": lds["lds_instr"],
                        "lds_conflict_share": lds["lds_bank_conflict_cycles"] / (us * 2400.0 * 256)})
        out[st] = row
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(x, q, L, eps, m, tol_mode="abs", label="full water box"):
    """The float64 oracle of the same computation (Alg. 2 in NumPy, oracle/fast.py), timed on this
    host: on all cores (the oracle's spreading and interpolation over particle chunks in one
    worker process per core, oracle/pool.py; the pool is started before the timed region) and on
    one thread; plus the single-core time of the plain n = 1000 system (m = 32, eps = 1e-6), by
    Alg. 2 and by the oracle's direct-sum route R2."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import direct, fast, params, pool as opool
    if tol_mode == "abs":
        p = params.choose(eps, L, m=m, q_l2=float(np.linalg.norm(q)), tol_mode="abs")
    else:
        p = params.choose(eps, L, m=m)
    cores = os.cpu_count() or 1
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        fast.fast_longrange(x, q, p, grad=True)
        dt1 = time.perf_counter() - t0
        ex = opool._pool(cores)
        try:
            list(ex.map(abs, range(cores)))          # workers started and idle
            t0 = time.perf_counter()
            opool.fast_longrange(x, q, p, pool=ex, nchunks=4 * cores)
            dtn = time.perf_counter() - t0
        finally:
            ex.shutdown()
        xc, qc, Lc = W.config("plain_fp64_n1000")
        pc = params.choose(1e-6, Lc, m=32)
        t0 = time.perf_counter()
        fast.fast_longrange(xc, qc, pc, grad=True)
        c1_fast = time.perf_counter() - t0
        t0 = time.perf_counter()
        direct.longrange_r2(xc, qc, Lc, pc.rc, pc.cs)
        c1_r2 = time.perf_counter() - t0
    n = len(q)
    return {"value": n / dtn, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": f"{label} (n={n}), one evaluation of oracle/fast.py (Alg. 2, float64 NumPy, phi and "
                      f"gradients) with its particle steps in {cores} worker processes, {dtn:.2f} s",
            "cpu_model": cpu_model(),
            "single_thread": {"value": n / dt1, "unit": "particles/s", "seconds": dt1},
            "plain_n1000_single_core": {"alg2_seconds": c1_fast, "direct_r2_seconds": c1_r2,
                                        "note": "n = 1000 uniform +-1, L = 1, eps = 1e-6, m = 32: oracle/fast.py "
                                                "and the direct route R2 of oracle/direct.py, one thread"}}


def bench_ensemble(steps: int, warmup: int):
    """Batched vs sequential: 256 independent neutral systems (n log-uniform in [500, 20000],
    L uniform in [0.5, 2], uniform positions, +-1 charges), each with its own eps = 1e-6
    parameters (Alg. 3, relative mode, 64-neighbour cutoff rule), float32 with float32 window
    arithmetic (the headline precision), phi + forces + energies. Batched: one plan over all
    systems, tiles from the autotuner, replayed as one HIP graph (and, for reference, called
    eagerly; and eagerly with float64 window arithmetic on the same tiles). Sequential: one
    default plan per system, called one after another."""
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
    prec = "fp32_arith"
    plan, tiles, report = autotune_batch(params, counts, X, Q, prec, targets=(None, 64, 256), reps=5)
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
    mixed = pw.BatchPlan(params, counts, "fp32", tiles=tiles)
    m_s = timed(lambda: mixed.compute(X, Q, phi=phi, force=F, energy=E), steps)
    mixed.close()
    singles = [pw.Plan(p, prec, n_max=c) for p, c in zip(params, counts)]
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
        "prec": prec,
        "batched_eager": {"value": n_total / e_s, "unit": "particles/s", "ms_per_step": e_s * 1e3},
        "batched_eager_fp32_mixed": {"value": n_total / m_s, "unit": "particles/s", "ms_per_step": m_s * 1e3},
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


def time_precisions(x, q, params_of, steps: int, warmup: int, with_total: bool, workload: str):
    """Both precisions of one workload: plan creation time, the timed steps, per-stage event
    times (a calibration pass before the timed region), the dominant stage's average launch time
    measured with events on the compute stream during the timed steps, and (with_total) the full
    Ewald sum with the real-space residual."""
    import numpy as np
    import torch
    import paper_2602_16591_amd as pw
    dev = torch.device("cuda:0")
    n = len(q)
    out = {}
    for prec in PRECISIONS:
        dt = torch.float64 if prec == "fp64" else torch.float32
        X = torch.as_tensor(x, dtype=dt, device=dev).contiguous()
        Q = torch.as_tensor(q, dtype=dt, device=dev).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = pw.Plan(params_of[prec], prec, n_max=n)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        phi = torch.empty(n, dtype=dt, device=dev)
        F = torch.empty((n, 3), dtype=dt, device=dev)
        E = torch.empty(1, dtype=torch.float64, device=dev)

        def step():
            plan.compute(X, Q, phi=phi, force=F, energy=E)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        # untimed calibration: average duration of every stage and of the whole call
        stage_ms = {}
        for st in STAGES + ["all"]:
            plan.timing_enable(st, 16)
            for _ in range(8):
                step()
            ms, calls = plan.timing_read()
            stage_ms[st] = ms / max(calls, 1)
        plan.timing_enable(None)
        dom = max(STAGES, key=stage_ms.get)
        plan.timing_enable(dom, steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        dom_ms_total, dom_calls = plan.timing_read()
        plan.timing_enable(None)
        p = params_of[prec]
        r = dict(elapsed=elapsed, dom=dom, dom_ms=dom_ms_total / max(dom_calls, 1), stage_ms=stage_ms, plan_s=plan_s,
                 phi=phi.double().cpu().numpy(), F=F.double().cpu().numpy(), E=float(E.cpu()[0]),
                 deg=pw.host_tables(p, prec)["deg"], elem=8 if prec == "fp64" else 4, m=p.m, P=p.P)
        if with_total:
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
            ksteps = max(10, steps // 4)
            for _ in range(ksteps):
                step_total()
            torch.cuda.synchronize()
            total_s = (time.perf_counter() - t1) / ksteps
            r["total"] = {"value": n / total_s, "unit": "particles/s", "ms_per_step": total_s * 1e3,
                          "local_overlapped_us": lms / max(lcalls, 1) * 1e3}
        plan.close()
        out[prec] = r
    return out


def leg_summary(r, n, steps, workload, prec):
    """A precision's figures for the JSON line."""
    ms = r["elapsed"] / steps * 1e3
    return {"value": n * steps / r["elapsed"], "unit": "particles/s", "ms_per_step": ms,
            "ms_per_step_excl_bin": ms - r["stage_ms"]["bin"],
            "call_us_event_timed": r["stage_ms"]["all"] * 1e3, "plan_create_s": r["plan_s"], "m": r["m"], "P": r["P"],
            "stage_us": {k: v * 1e3 for k, v in r["stage_ms"].items() if k != "all"},
            "kernels": kernel_rooflines(r["stage_ms"], n, r["m"], r["P"], r["deg"], r["elem"], prec, workload)}


def roofline_of(r, n, workload, prec):
    kind, work = stage_work(r["dom"], n, r["m"], r["P"], r["deg"], r["elem"])
    secs = r["dom_ms"] * 1e-3
    if kind in ("alu", "mfma"):
        # the particle kernels' arithmetic: float32 on the float32 arithmetic path (the spread on
        # the float32 matrix cores), float64 otherwise (the float64 matrix-core peak on MI355X
        # equals the float64 vector rate)
        peak = peak_tflops(prec)
        achieved = work / secs / 1e12
        roof = {"bound": kind, "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        achieved = work / secs / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof["traffic"] = measured_traffic(r["dom"], prec, workload)
    roof.update({"kernel": r["dom"], "avg_launch_us": r["dom_ms"] * 1e3, "work_per_launch": work})
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("water_box_n30000", "uniform_n1e6"), default="water_box_n30000",
                    help="the headline workload: the water box (default) or n = 1e6 uniform (float32 at eps 1e-6 "
                         "on 128^3, float64 at eps 1e-10 with the same r_c)")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential ensemble")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the split/window comparison at the paper's resolutions")
    ap.add_argument("--no-large", action="store_true",
                    help="with the water box as headline: skip the n = 1e6 legs")
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

    def water_inputs():
        x, q, L = W.config("water_n30000")
        p = pw.choose_params(1e-6, L, m=64, q_l2=float(np.linalg.norm(q)), tol_mode="abs")
        return x, q, L, {"fp32": p, "fp64": p}

    def large_inputs():
        x, q, L = W.config("uniform_n1e6")
        p = pw.choose_params(1e-6, L, m=128)
        return x, q, L, {"fp32": p, "fp64": pw.choose_params(1e-10, L, rc=p.rc)}

    water = args.workload == "water_box_n30000"
    x, q, L, params_of = water_inputs() if water else large_inputs()
    # both precisions get the same float32-representable inputs, so the float32/float64
    # comparison isolates arithmetic error from input quantisation
    x = x.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    n = len(q)
    params_of["fp32_arith"] = params_of["fp32"]
    res = time_precisions(x, q, params_of, args.steps, args.warmup, with_total=water, workload=args.workload)
    r, rmix, r64 = res["fp32_arith"], res["fp32"], res["fp64"]
    p32, p64 = params_of["fp32"], params_of["fp64"]
    if water:
        config = {"workload": "water_box_n30000", "n": n, "L_nm": L, "eps": 1e-6, "tol_mode": "abs", "m": p32.m,
                  "P": p32.P, "rc_nm": p32.rc, "parallelism": "single GPU"}
    else:
        config = {"workload": "uniform_n1e6", "n": n, "L": L, "eps": 1e-6, "tol_mode": "rel", "m": p32.m, "P": p32.P,
                  "rc": p32.rc, "fp64": {"eps": 1e-10, "m": p64.m, "P": p64.P}, "parallelism": "single GPU"}
    leg32 = leg_summary(r, n, args.steps, args.workload, "fp32_arith")
    legmix = leg_summary(rmix, n, args.steps, args.workload, "fp32")
    leg64 = leg_summary(r64, n, args.steps, args.workload, "fp64")
    keys = ("value", "unit", "ms_per_step", "ms_per_step_excl_bin", "stage_us", "plan_create_s", "m", "P")

    def diff(a, b):
        return {"phi_rel_l2": float(np.linalg.norm(a["phi"] - b["phi"]) / np.linalg.norm(b["phi"])),
                "phi_abs_rms": float(np.sqrt(np.mean((a["phi"] - b["phi"]) ** 2))),
                "force_rel_l2": float(np.linalg.norm(a["F"] - b["F"]) / np.linalg.norm(b["F"])),
                "energy_rel": abs(a["E"] - b["E"]) / abs(b["E"])}

    out = {
        "metric": METRIC, "value": leg32["value"], "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": config,
        "roofline": roofline_of(r, n, args.workload, "fp32_arith"),
        "precision_note": "headline: float32 inputs, grids and outputs with float32 window values, products and sums in "
                          "spreading (float32 matrix cores) and interpolation (plan precision fp32_arith); fp32_mixed: "
                          "float32 storage with float64 arithmetic; fp64: float64 throughout",
        "ms_per_step_excl_bin": leg32["ms_per_step_excl_bin"],
        "plan_create_s": {"fp32_arith": r["plan_s"], "fp32_mixed": rmix["plan_s"], "fp64": r64["plan_s"]},
        "stage_us_fp32": leg32["stage_us"],
        "fp32_mixed": {k: legmix[k] for k in keys},
        "fp64": {k: leg64[k] for k in keys},
        "kernels_fp32": leg32["kernels"],
        "kernels_fp32_mixed": legmix["kernels"],
        "kernels_fp64": leg64["kernels"],
        "fp32_vs_fp64": diff(r, r64),
        "fp32_mixed_vs_fp64": diff(rmix, r64),
    }
    if water:
        out["total_ewald"] = {"note": "phi_far + phi_local + phi_self (real-space residual on the GPU), same workload; "
                                      "local_overlapped_us: the residual's span on its own stream, which it shares "
                                      "with the long-range kernels running at the same time",
                              "fp32": r["total"], "fp32_mixed": rmix["total"], "fp64": r64["total"]}
        if not args.no_large:
            # the n = 1e6 system, both precisions, as extra keys (the headline stays the water box)
            xl, ql, Ll, pl = large_inputs()
            pl["fp32_arith"] = pl["fp32"]
            xl = xl.astype(np.float32).astype(np.float64)
            ql = ql.astype(np.float32).astype(np.float64)
            ksteps = max(10, min(args.steps, 50))
            resl = time_precisions(xl, ql, pl, ksteps, max(2, min(args.warmup, 5)), with_total=False,
                                   workload="uniform_n1e6")
            out["uniform_n1e6"] = {
                "note": "n = 1e6 uniform charges U[-1,1] minus the mean, L = 1; float32 at eps = 1e-6 (relative) on "
                        "128^3, float64 at eps = 1e-10 with the same r_c; phi + forces + energy",
                "steps": ksteps, "rc": pl["fp32"].rc,
                "fp32": leg_summary(resl["fp32_arith"], len(ql), ksteps, "uniform_n1e6", "fp32_arith"),
                "fp32_mixed": leg_summary(resl["fp32"], len(ql), ksteps, "uniform_n1e6", "fp32"),
                "fp64": leg_summary(resl["fp64"], len(ql), ksteps, "uniform_n1e6", "fp64"),
                "roofline_fp32": roofline_of(resl["fp32_arith"], len(ql), "uniform_n1e6", "fp32_arith"),
                "fp32_mixed_vs_fp32_rel_l2_phi": float(np.linalg.norm(resl["fp32_arith"]["phi"] - resl["fp32"]["phi"]) /
                                                        np.linalg.norm(resl["fp32"]["phi"])),
            }
            del xl, ql
    if not args.no_batched:
        out["batched"] = bench_ensemble(max(5, min(args.steps, 50)), max(2, min(args.warmup, 5)))
    if not args.no_comparison:
        out["comparison"] = bench_comparison(max(5, min(args.steps, 30)), max(2, min(args.warmup, 5)))
    if not args.no_cpu_baseline:
        if water:
            out["cpu_baseline"] = cpu_baseline(x, q, L, 1e-6, p32.m)
        else:
            out["cpu_baseline"] = cpu_baseline(x, q, L, 1e-6, p32.m, tol_mode="rel", label="uniform n = 1e6")
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

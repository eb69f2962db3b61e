"""Measured choice of the tile (bin) edge of binning, spreading and interpolation.

Particles are binned by tiles of B^3 grid cells; one workgroup handles a tile with an LDS copy
of the S^3 points its supports touch, S = B + 2 ceil(P/2) - 1. Small tiles give more
workgroups but more halo points to clear, flush and load per particle; large tiles give fewer,
longer workgroups and, through their LDS footprint, fewer resident workgroups per compute
unit. The best edge depends on the particle density, P, the grid size and the precision, so
it is measured: every candidate runs as a captured graph (the way it is used) and is timed
with HIP events; the fastest is kept. Results can be cached in a dict or a JSON file, keyed
by the problem's shape.
"""
from __future__ import annotations

import json
import math
import os

from . import BatchPlan, Plan, _prec

DENSITY_TARGETS = (None, 32, 64, 128, 256, 1024)  # None: tile edge 8 everywhere (spreading by columns)
SINGLE_TILES = (4, 5, 6, 7, 8, 9, 10, 12)


def tile_for_density(m: int, n: int, target: float) -> int:
    """Smallest tile edge (>= 4, <= m) with about `target` particles per tile on average."""
    if n <= 0:
        return min(m, 8)
    b = math.ceil((target * m ** 3 / n) ** (1.0 / 3.0) - 1e-9)
    return int(max(4, min(m, b)))


def time_replays(runner, reps: int = 10, warmup: int = 3) -> float:
    """Median milliseconds of `reps` replays of a CapturedCompute (HIP events, current stream)."""
    import torch
    for _ in range(warmup):
        runner()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        runner()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def _load(cache):
    if isinstance(cache, (str, os.PathLike)):
        if os.path.exists(cache):
            with open(cache) as f:
                return json.load(f)
        return {}
    return cache if cache is not None else {}


def _store(cache, table):
    if isinstance(cache, (str, os.PathLike)):
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


def _key(kind, prec, params, counts):
    shape = ";".join(f"{p.m},{p.P},{round(p.L, 12)},{c}" for p, c in zip(params, counts))
    return f"{kind}|{_prec(prec)}|{shape}"


def autotune_batch(params, counts, pos, q, prec="fp32", targets=DENSITY_TARGETS, reps: int = 10, cache=None,
                   **compute_kw):
    """Picks per-system tile edges for a batch. Each candidate is a particles-per-tile target
    turned into one edge per system (tile_for_density), or None for edge 8 everywhere (where
    spreading runs by register columns); the candidate with the fastest graph replay wins.
    Returns (BatchPlan with the chosen tiles, tiles, report) where report lists (target, tiles,
    ms) per candidate (empty when the cache answered)."""
    params, counts = list(params), [int(c) for c in counts]
    table = _load(cache)
    key = _key("batch", prec, params, counts)
    if key in table:
        tiles = table[key]["tiles"]
        return BatchPlan(params, counts, prec, tiles=tiles), tiles, []
    P = max(p.P for p in params)
    report, best = [], None
    seen = set()
    for t in targets:
        tiles = [min(8, p.m) if t is None else tile_for_density(p.m, c, t) for p, c in zip(params, counts)]
        if tuple(tiles) in seen:
            continue
        seen.add(tuple(tiles))
        plan = BatchPlan(params, counts, prec, tiles=tiles)
        runner = plan.graph(pos, q, **compute_kw)
        ms = time_replays(runner, reps)
        report.append((t, plan.tiles, ms))
        if best is None or ms < best[0]:
            best = (ms, plan.tiles)
        del runner
        plan.close()
    tiles = best[1]
    table[key] = {"tiles": tiles, "ms": best[0], "P": P}
    _store(cache, table)
    return BatchPlan(params, counts, prec, tiles=tiles), tiles, report


def autotune_plan(params, pos, q, prec="fp32", tiles=SINGLE_TILES, reps: int = 10, cache=None, **compute_kw):
    """Picks the tile edge of a single-system plan for n = len(pos) particles. Returns
    (Plan with the chosen tile, tile, report of (tile, ms))."""
    n = int(pos.shape[0])
    table = _load(cache)
    key = _key("single", prec, [params], [n])
    if key in table:
        t = table[key]["tile"]
        return Plan(params, prec, n_max=n, tile=t), t, []
    report, best, seen = [], None, set()
    for t in tiles:
        if t > params.m:
            continue
        plan = Plan(params, prec, n_max=n, tile=t)
        if plan.tile in seen:       # reduced to an edge already measured (LDS limits)
            plan.close()
            continue
        seen.add(plan.tile)
        runner = plan.graph(pos, q, **compute_kw)
        ms = time_replays(runner, reps)
        report.append((plan.tile, ms))
        if best is None or ms < best[0]:
            best = (ms, plan.tile)
        del runner
        plan.close()
    table[key] = {"tile": best[1], "ms": best[0]}
    _store(cache, table)
    return Plan(params, prec, n_max=n, tile=best[1]), best[1], report

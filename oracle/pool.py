"""The float64 oracle of Alg. 2 on large systems, its particle steps spread over worker
processes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``); also times the oracle on all host cores
for the benchmark's CPU baseline.

Spreading (step 1) is linear in the charges, so the grid of all particles is the sum of the
grids of disjoint chunks; interpolation (step 5) is independent per particle. This module calls
the oracle's own step functions (oracle/fast.py: spread, scaling, interpolate, and NumPy's FFT
as fast_longrange does) on chunks in spawned processes that import only NumPy and the oracle;
it adds no arithmetic of its own beyond the sum of the chunk grids. A CPU test checks that it
reproduces fast.fast_longrange to rounding.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _spread(args):
    from oracle import fast
    x, q, o = args
    return fast.spread(x, q, o)


def _interp(args):
    from oracle import fast
    b, x, o, grad = args
    return fast.interpolate(b, x, o, grad=grad)


def workers(limit: int = 8) -> int:
    return max(1, min(limit, os.cpu_count() or 1))


def _chunks(n, k):
    edges = np.linspace(0, n, k + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def _pool(nworkers: int | None = None):
    return ProcessPoolExecutor(max_workers=nworkers or workers(), mp_context=mp.get_context("spawn"))


def spread(x, q, o, pool=None, nchunks=16):
    """fast.spread(x, q, o) as the sum of the spreads of particle chunks."""
    own = pool is None
    pool = pool or _pool()
    try:
        parts = pool.map(_spread, [(x[a:b], q[a:b], o) for a, b in _chunks(len(q), nchunks)])
        a = np.zeros((o.m, o.m, o.m))
        for g in parts:
            a += g
        return a
    finally:
        if own:
            pool.shutdown()


def interpolate(b, x, o, grad=True, pool=None, nchunks=16):
    """fast.interpolate(b, x, o) evaluated on particle chunks."""
    own = pool is None
    pool = pool or _pool()
    try:
        res = list(pool.map(_interp, [(b, x[a:c], o, grad) for a, c in _chunks(len(x), nchunks)]))
        phi = np.concatenate([r[0] for r in res]) if res else np.zeros(0)
        g = np.concatenate([r[1] for r in res]) if (res and grad) else None
        return phi, g
    finally:
        if own:
            pool.shutdown()


def fast_longrange(x, q, o, return_grids=False, nworkers=None, nchunks=16, pool=None):
    """fast.fast_longrange(x, q, o) (phi_far + phi_self and grad phi_far) with steps 1 and 5 over
    chunks in worker processes (a pool of `nworkers`, or the `pool` given); steps 2-4 as in
    fast.fast_longrange."""
    from oracle import fast
    from oracle.direct import self_term
    x = np.mod(np.asarray(x, dtype=np.float64), o.L)
    q = np.asarray(q, dtype=np.float64)
    own = pool is None
    pool = pool or _pool(nworkers)
    try:
        a = spread(x, q, o, pool=pool, nchunks=nchunks)
        ahat = np.fft.ifftn(a) * o.m ** 3
        b = np.fft.fftn(fast.scaling(o, ball=True) * ahat).real
        del ahat
        phi, g = interpolate(b, x, o, pool=pool, nchunks=nchunks)
    finally:
        if own:
            pool.shutdown()
    phi = phi + self_term(q, o.rc, o.cs)
    if return_grids:
        return phi, g, dict(a=a, b=b)
    return phi, g

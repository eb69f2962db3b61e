"""Per-particle support sums of tests/elementwise.py over particle chunks in worker processes
(test infrastructure); the oracle's own chunked steps are in oracle/pool.py."""
from __future__ import annotations

import numpy as np

from oracle.pool import _chunks, _pool, fast_longrange, interpolate, spread  # noqa: F401


def _abs_sum(args):
    import elementwise
    b, x, o = args
    return elementwise.support_abs_sum(b, x, o)


def support_abs_sum(b, x, o, pool=None, nchunks=16):
    own = pool is None
    pool = pool or _pool()
    try:
        return np.concatenate(list(pool.map(_abs_sum, [(b, x[a:c], o) for a, c in _chunks(len(x), nchunks)])))
    finally:
        if own:
            pool.shutdown()

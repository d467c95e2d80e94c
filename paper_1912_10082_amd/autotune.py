"""Measurement-driven choice of the batch executor's concurrency.

How many solves should run at once depends on the mix: small grids leave most
of the 256 compute units idle and gain from many concurrent solves, large
grids fill the chip alone and lose to contention.  ``tune_workers`` times
``sts_pool_solve`` on a probe subset of the batch for each candidate worker
count and returns the fastest.  Every candidate solves the same probe from
scratch (``restart=1``), after one untimed pass that performs the problems'
first-solve allocations, so the comparison is like for like.
"""
from __future__ import annotations

import time

from .binding import Pool

DEFAULT_CANDIDATES = (1, 2, 4, 8)


def probe_subset(problems, size: int) -> list:
    """Every k-th problem, so that the probe spans the batch's mix."""
    if len(problems) <= size:
        return list(problems)
    stride = len(problems) / float(size)
    return [problems[int(i * stride)] for i in range(size)]


def tune_workers(problems, candidates=DEFAULT_CANDIDATES, probe: int = 24, repeats: int = 1,
                 **opts) -> tuple:
    """Return (best worker count, {workers: seconds}) for ``problems``.

    ``opts`` are the solve options of the real batch (``restart`` is forced
    to 1).  Ties go to the smaller worker count.
    """
    sub = probe_subset(problems, probe)
    opts = dict(opts, restart=1)
    timings = {}
    with Pool(max(candidates)) as warm:
        warm.solve(sub, **opts)
    for w in candidates:
        with Pool(w) as pool:
            best = None
            for _ in range(repeats):
                t0 = time.perf_counter()
                infos = pool.solve(sub, **opts)
                dt = time.perf_counter() - t0
                bad = [d for d in infos if d["status"] != "STS_OK"]
                if bad:
                    raise RuntimeError(f"probe solve failed with {w} workers: {bad[0]}")
                best = dt if best is None else min(best, dt)
        timings[w] = best
    chosen = min(sorted(timings), key=lambda w: timings[w])
    return chosen, timings

"""Measurement-driven choice of the batch executor's schedule.

How many solves should run at once depends on the mix: small grids leave most
of the 256 compute units idle and gain from many concurrent solves (while one
worker's stream waits on a host decision, the others have work queued), large
grids fill the chip alone and lose to contention.  How far the inner solves
may be relaxed as the residual falls (``inner_relax``, inexact Krylov) trades
inner iterations against extra outer blocks, and the best point depends on
the grids too.  ``tune`` times ``sts_pool_solve`` on a probe subset of the
batch for every (worker count, relaxation) pair and returns the fastest;
``tune_workers`` searches the worker count alone.  Every candidate solves the
same probe from scratch (``restart=1``), after one untimed pass that performs
the problems' first-solve allocations, so the comparison is like for like.
"""
from __future__ import annotations

import itertools
import time

from .binding import Pool

DEFAULT_CANDIDATES = (1, 2, 4, 8, 16, 32)
DEFAULT_RELAX = (1, 2)


def probe_subset(problems, size: int) -> list:
    """Every k-th problem, so that the probe spans the batch's mix."""
    if len(problems) <= size:
        return list(problems)
    stride = len(problems) / float(size)
    return [problems[int(i * stride)] for i in range(size)]


def _time_probe(sub, workers: int, repeats: int, opts: dict) -> float:
    with Pool(workers) as pool:
        best = None
        for _ in range(repeats):
            t0 = time.perf_counter()
            infos = pool.solve(sub, **opts)
            dt = time.perf_counter() - t0
            bad = [d for d in infos if d["status"] != "STS_OK"]
            if bad:
                raise RuntimeError(f"probe solve failed with {workers} workers: {bad[0]}")
            best = dt if best is None else min(best, dt)
    return best


def tune(problems, candidates=DEFAULT_CANDIDATES, relax=DEFAULT_RELAX, probe: int = 32,
         repeats: int = 1, **opts) -> tuple:
    """Return ((workers, inner_relax), {(workers, inner_relax): seconds}).

    ``opts`` are the solve options of the real batch (``restart`` is forced
    to 1, ``inner_relax`` is searched).  Ties go to fewer workers, then to
    the smaller relaxation exponent.
    """
    sub = probe_subset(problems, probe)
    base = dict(opts, restart=1)
    with Pool(max(candidates)) as warm:
        warm.solve(sub, **dict(base, inner_relax=relax[0]))
    timings = {}
    for w, j in itertools.product(candidates, relax):
        timings[(w, j)] = _time_probe(sub, w, repeats, dict(base, inner_relax=j))
    chosen = min(sorted(timings), key=lambda key: timings[key])
    return chosen, timings


def tune_workers(problems, candidates=DEFAULT_CANDIDATES, probe: int = 24, repeats: int = 1,
                 **opts) -> tuple:
    """Return (best worker count, {workers: seconds}) for ``problems``.

    ``opts`` are the solve options of the real batch (``restart`` is forced
    to 1).  Ties go to the smaller worker count.
    """
    sub = probe_subset(problems, probe)
    opts = dict(opts, restart=1)
    with Pool(max(candidates)) as warm:
        warm.solve(sub, **opts)
    timings = {w: _time_probe(sub, w, repeats, opts) for w in candidates}
    chosen = min(sorted(timings), key=lambda w: timings[w])
    return chosen, timings

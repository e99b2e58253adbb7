"""Batch-width autotuner: picks B (the labels popped per step, the paper's
NUM_POP) for a list of queries on one graph by measuring the library itself.

A wider batch gives every step more independent work (the GPU's parallelism)
at the cost of labels popped beyond the sequential order (the paper's work
efficiency, Section 4); which side wins depends on the graph, the objective
count and the queries.  The tuner solves a seeded sample of the queries with
``mos_solve_batch`` at each candidate width and keeps the fastest width.  The
library caches engines per graph by (slot count, width, paths or not, ...), so
the first call at each width, untimed, is the same call as the timed ones:
the timed calls then reuse its engine and time only the search.  Every width
must give the same fronts (the result does not depend on the pop order); a
disagreement raises.
"""
from __future__ import annotations

import time

import numpy as np

from . import MOS_OK, MosError, mos_solve_batch

DEFAULT_WIDTHS = (256, 1024, 4096, 16384)


def tune_batch_width(graph, starts, goals, n_objectives=None, widths=DEFAULT_WIDTHS,
                     sample: int = 16, seed: int = 0, repeats: int = 1, costs_only: bool = True,
                     **opts) -> dict:
    """Returns {"batch_width": B, "seconds": {B: wall seconds of the sample},
    "sample": number of queries timed}.  `opts` are passed to every solve
    (mem_budget, max_slots, ...).  The sample should look like the real call:
    the engine's slot count follows the number of queries, and with
    ``costs_only=False`` the tuned engine is the one a later call with paths
    reuses."""
    starts = np.ascontiguousarray(starts, dtype=np.int32)
    goals = np.ascontiguousarray(goals, dtype=np.int32)
    nq = starts.shape[0]
    if nq == 0 or not widths:
        raise ValueError("need at least one query and one width")
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(nq, size=min(sample, nq), replace=False))
    S, T = starts[pick], goals[pick]
    D = None if n_objectives is None else np.ascontiguousarray(n_objectives, np.int32)[pick]
    seconds, fronts = {}, None
    for B in widths:
        mos_solve_batch(graph, S, T, D, batch_width=B, costs_only=costs_only, **opts)
        best = float("inf")
        for _ in range(max(1, repeats)):
            t0 = time.perf_counter()
            res = mos_solve_batch(graph, S, T, D, batch_width=B, costs_only=costs_only, **opts)
            best = min(best, time.perf_counter() - t0)
        if any(st != MOS_OK for st, _ in res):
            raise MosError(next(st for st, _ in res if st != MOS_OK), f"autotune at B={B}")
        got = [r.costs for _, r in res]
        if fronts is None:
            fronts = got
        elif not all(np.array_equal(a, b) for a, b in zip(fronts, got)):
            raise RuntimeError(f"fronts differ between batch widths (B={B})")
        seconds[int(B)] = best
    bw = min(seconds, key=lambda b: (seconds[b], b))
    return {"batch_width": bw, "seconds": seconds, "sample": int(len(pick))}

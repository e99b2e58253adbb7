"""Shared test helpers: independent checks of a front (used for both sides)."""
from __future__ import annotations

import numpy as np


def sort_lex(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64)
    if a.size == 0:
        return a.reshape(0, a.shape[1] if a.ndim == 2 else 0)
    return a[np.lexsort(a.T[::-1])]


def is_antichain(front: np.ndarray) -> bool:
    """No vector weakly dominates another (distinct rows, none <= another)."""
    f = np.asarray(front, dtype=np.int64)
    for i in range(f.shape[0]):
        le = np.all(f <= f[i], axis=1)
        le[i] = False
        if le.any():
            return False
    return True


def path_cost(g, s, t, arcs, d) -> np.ndarray:
    """Re-sum a path given as CSR arc ids; checks it is a connected s->t walk."""
    src = g.arc_sources()
    cur = s
    tot = np.zeros(d, dtype=np.int64)
    for e in arcs:
        assert src[e] == cur, "path is not connected"
        tot += g.cost[e, :d]
        cur = int(g.col[e])
    assert cur == t, "path does not end at the goal"
    return tot


def check_paths(g, s, t, costs, paths, d):
    for c, p in zip(costs, paths):
        assert np.array_equal(path_cost(g, s, t, p, d), np.asarray(c, dtype=np.int64))

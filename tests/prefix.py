"""Checks of a GPU front against the oracle when either side may hold only an
exact prefix of the front, and the necessary conditions that every complete
front must meet (test helpers; the oracle supplies every reference value).

Both kinds of prefix are exact: the oracle's early-stopped front is the final
front below the F of its smallest open label (lexicographic order); the GPU's
step-limited or so-far front is the final front below its bound on the first
objective.  Inside the intersection of the two ranges both must therefore be
the same set, entry for entry.
"""
import itertools

import numpy as np

import oracle


def in_range(y, gpu_f1, ora_bound):
    """y lies below the GPU bound on objective 0 (None: complete) and below the
    oracle's lexicographic bound (None: complete)."""
    if gpu_f1 is not None and not y[0] < gpu_f1:
        return False
    if ora_bound is not None and not oracle.lex_less(y, ora_bound):
        return False
    return True


def _select(rows, gpu_f1, ora_bound):
    rows = np.asarray(rows, dtype=np.int64)
    if rows.size == 0:
        return []
    keep = np.ones(rows.shape[0], dtype=bool)
    if gpu_f1 is not None:
        keep &= rows[:, 0] < gpu_f1
    if ora_bound is not None:
        keep &= rows[:, 0] <= ora_bound[0]  # cheap filter, then the exact test
    return [tuple(int(x) for x in y) for y in rows[keep] if in_range(y, gpu_f1, ora_bound)]


def compare_prefix(gpu_rows, gpu_f1, ora_rows, ora_bound):
    """Assert both sides agree on the common range; returns the number of
    entries compared."""
    a = _select(gpu_rows, gpu_f1, ora_bound)
    b = _select(ora_rows, gpu_f1, ora_bound)
    assert a == b, (len(a), len(b), next(((i, x, y) for i, (x, y) in enumerate(zip(a, b))
                                           if x != y), None))
    return len(a)


def lex_min(front, perm):
    f = np.asarray(front, dtype=np.int64)
    return tuple(int(x) for x in f[np.lexsort(f[:, list(perm)].T[::-1])[0]])


def necessary_conditions(g, s, t, d, front, n_weights=6, seed=0, perms=None):
    """A complete front of s->t over the first d objectives: sorted, mutually
    non-dominated, its ideal point, its lexicographic extremes for every
    objective order (or the given ones) and its supported minima for random
    positive weights are those of single-criterion shortest paths."""
    f = np.asarray(front, dtype=np.int64).reshape(-1, d)
    assert f.shape[0] > 0
    assert oracle.first_dominated(f) == -1
    h = oracle.heuristic(g, t, d)
    assert np.array_equal(f.min(axis=0), h[:, s]), "ideal point"
    for perm in (perms if perms is not None else itertools.permutations(range(d))):
        assert lex_min(f, perm) == oracle.lex_dijkstra(g, s, t, perm), perm
    rng = np.random.default_rng(seed)
    for _ in range(n_weights):
        w = rng.integers(1, 64, d)
        assert int((f @ w).min()) == int(oracle.scalar_dijkstra(g, s, w)[t]), w

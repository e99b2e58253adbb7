"""Pins of the oracle's large-graph checks against brute force on tiny graphs.

The checks that stay cheap when the exact search does not finish (paper,
Section 3 defines the front; the facts below follow from that definition):
  * oracle.lex_dijkstra: for every order of the objectives, the cost of the
    lexicographically shortest path is the lexicographically smallest front
    vector under that order;
  * oracle.scalar_dijkstra: for positive weights w, the shortest distance
    under the arc cost w . c is the smallest w . y over the front;
  * the prefix of an early-stopped search: the oracle's goal front when it is
    stopped after any number of extractions equals the exact front restricted
    to the vectors lexicographically below the F of the smallest label left in
    OPEN (with OPEN in lexicographic order and a consistent heuristic, goal
    labels leave OPEN in increasing cost order and none of them is dominated
    later).
Each is compared here with the minimal set of all simple-path costs
enumerated by DFS, never with another run of the same code.
"""
import itertools

import numpy as np
import pytest

import gen
import oracle
from helpers import sort_lex
from test_oracle_pins import MODES, brute_front


def lex_min(front, perm):
    f = np.asarray(front)[:, list(perm)]
    return tuple(int(x) for x in np.asarray(front)[np.lexsort(f.T[::-1])[0]])


CASES = [(gen.random_small(8, 20, 1 + seed % 4, seed=seed), 1 + seed % 4, st)
         for seed in range(12) for st in [(0, 7), (2, 5), (6, 1)]]
CASES += [(gen.grid_uniform(r, c, d, 0, 5, seed=r * 10 + c), d, (0, r * c - 1))
          for r, c, d in [(3, 3, 3), (3, 4, 2), (4, 4, 3), (4, 5, 2)]]


@pytest.mark.parametrize("i", range(len(CASES)))
def test_lex_dijkstra_is_the_lexicographic_extreme(i):
    g, d, (s, t) = CASES[i]
    ref = brute_front(g, s, t, d)
    for perm in itertools.permutations(range(d)):
        got = oracle.lex_dijkstra(g, s, t, perm)
        if ref.shape[0] == 0:
            assert got is None
        else:
            assert got == lex_min(ref, perm), (i, perm)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_scalar_dijkstra_is_the_supported_minimum(i):
    g, d, (s, t) = CASES[i]
    ref = brute_front(g, s, t, d)
    rng = np.random.default_rng(i)
    for _ in range(6):
        w = rng.integers(1, 20, d)
        dist = oracle.scalar_dijkstra(g, s, w)[t]
        if ref.shape[0] == 0:
            assert dist == np.iinfo(np.int64).max
        else:
            assert dist == int((ref @ w).min()), (i, w)


def test_scalar_dijkstra_counts_zero_cost_arcs():
    # a zero-cost arc must be usable (not dropped like an absent entry)
    g = gen.from_arcs(3, [0, 1, 0], [1, 2, 2], np.array([[0, 0], [0, 0], [5, 5]]))
    assert oracle.scalar_dijkstra(g, 0, [1, 1])[2] == 0
    assert oracle.lex_dijkstra(g, 0, 2, (1, 0)) == (0, 0)


@pytest.mark.parametrize("i", range(0, len(CASES), 3))
@pytest.mark.parametrize("mode", MODES[:4])
def test_early_stopped_front_is_the_exact_prefix(i, mode):
    g, d, (s, t) = CASES[i]
    ref = brute_front(g, s, t, d)
    full = oracle.solve(g, s, t, d, flags=mode)
    stops = 0
    for limit in range(1, full.stats["pops"] + full.stats["killed"] + 1):
        r = oracle.solve(g, s, t, d, flags=mode, pop_limit=limit)
        if r.status == "ok":
            break
        assert r.status == "time limit" and r.open_min is not None
        stops += 1
        bound, rows = oracle.prefix_bound(r)
        want = [y for y in ref if oracle.lex_less(y, bound)]
        assert np.array_equal(sort_lex(np.array(want, np.int64).reshape(-1, d)), rows), (i, limit)
        # nothing found so far is ever removed again
        got = {tuple(int(x) for x in y) for y in r.costs}
        assert got <= {tuple(int(x) for x in y) for y in ref}
    assert stops > 0 or full.stats["pops"] <= 1


@pytest.mark.parametrize("seed", [0, 5])
def test_early_stopped_front_prefix_on_a_grid_query(seed):
    # a 32x32 query with a front of thousands of vectors: the full run is the
    # reference here, and it is itself pinned by the supported and extreme points
    g, s, t = gen.config1(seed)
    full = oracle.solve(g, s, t, 3, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
    for perm in itertools.permutations(range(3)):
        assert oracle.lex_dijkstra(g, s, t, perm) == lex_min(full.costs, perm)
    for limit in (500, 5000, 20000, 60000):
        r = oracle.solve(g, s, t, 3, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN, pop_limit=limit)
        if r.status == "ok":
            continue
        bound, rows = oracle.prefix_bound(r)
        want = np.array([y for y in full.costs if oracle.lex_less(y, bound)], np.int64).reshape(-1, 3)
        assert np.array_equal(want, rows), limit


@pytest.mark.parametrize("seed", range(6))
def test_first_dominated_is_the_antichain_test(seed):
    from helpers import is_antichain

    rng = np.random.default_rng(seed)
    for d in (2, 3, 5):
        for _ in range(40):
            a = sort_lex(np.unique(rng.integers(0, 6, (rng.integers(1, 12), d)), axis=0))
            got = oracle.first_dominated(a)
            assert (got == -1) == is_antichain(a)
            if got >= 0:
                # the reported row really is weakly dominated by an earlier one
                assert np.any(np.all(a[:got] <= a[got], axis=1))
    assert oracle.first_dominated(np.array([[1, 2], [1, 2]])) == 1  # duplicates
    assert oracle.first_dominated(np.array([[2, 1], [1, 2]])) == -2  # not ascending

"""GPU path vs the CPU oracle: exact (bit-identical) fronts, through the C ABI."""
import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths, is_antichain, sort_lex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def _front(mos, g, s, t, d=None, **kw):
    G = mos.Graph.from_gen(g)
    r = mos.mos_solve(G, s, t, n_objectives=d or 0, **kw)
    return r


@pytest.mark.parametrize("seed", [0, 1])
def test_heuristic_matches_dijkstra(mos, seed):
    g, s, t = gen.config1(seed)
    G = mos.Graph.from_gen(g)
    h = mos.mos_heuristic(G, t)
    ref = oracle.heuristic(g, t)
    ref32 = np.where(ref == oracle.INF, np.iinfo(np.int32).max, ref).astype(np.int32)
    assert np.array_equal(h, ref32)


def test_heuristic_unreachable_nodes(mos):
    g = gen.random_small(12, 14, 3, seed=5, self_loops=True)
    G = mos.Graph.from_gen(g)
    for goal in range(g.n):
        h = mos.mos_heuristic(G, goal)
        ref = oracle.heuristic(g, goal)
        ref32 = np.where(ref == oracle.INF, np.iinfo(np.int32).max, ref).astype(np.int32)
        assert np.array_equal(h, ref32), goal


@pytest.mark.parametrize("B", [1, 7, 64, 256])
def test_small_grid_front(mos, B):
    g = gen.grid_uniform(8, 8, 3, 1, 10, seed=3)
    r = _front(mos, g, 0, g.n - 1, batch_width=B)
    ref = oracle.solve(g, 0, g.n - 1)
    assert np.array_equal(r.costs.astype(np.int64), ref.costs)
    check_paths(g, 0, g.n - 1, r.costs, r.paths, 3)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_random_graphs(mos, seed):
    d = 1 + seed % 4
    g = gen.random_small(9, 24, d, seed=seed)
    for s, t in [(0, 8), (3, 3), (5, 1)]:
        r = _front(mos, g, s, t, batch_width=4)
        ref = oracle.solve(g, s, t)
        assert ref.status == "ok"
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, s, t)
        check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config1_front(mos, seed):
    g, s, t = gen.config1(seed)
    r = _front(mos, g, s, t, batch_width=256)
    ref = oracle.solve(g, s, t, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
    assert r.costs.shape == ref.costs.shape
    assert np.array_equal(r.costs.astype(np.int64), ref.costs)
    assert is_antichain(r.costs)
    check_paths(g, s, t, r.costs, r.paths, 3)

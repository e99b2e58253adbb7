"""Relaxed OPEN order (pop_order="generation": the B oldest labels by the step
that generated them, a first-in first-out queue of generations instead of the
lexicographic priority queue).  The paper compares the two orders (Section 7.1);
any order reaches the same front, so the same oracle decides, bit for bit.
The order changes only the work: the test also records labels popped against
the lexicographic order's."""
import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths

pytestmark = pytest.mark.gpu

FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


@pytest.mark.parametrize("B", [256, 4096])
def test_grid_fronts_in_generation_order(mos, B):
    for seed in (0, 3):
        g, s, t = gen.config1(seed)
        G = mos.Graph.from_gen(g)
        r = mos.mos_solve(G, s, t, batch_width=B, pop_order="generation", mem_budget=1 << 30)
        ref = oracle.solve(g, s, t, 3, flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, B)
        check_paths(g, s, t, r.costs, r.paths, 3)


@pytest.mark.parametrize("seed", range(8))
def test_random_multigraphs_in_generation_order(mos, seed):
    d = 1 + seed % 4
    g = gen.random_small(9, 26, d, seed=seed)
    G = mos.Graph.from_gen(g)
    for s, t in [(0, 8), (3, 5), (7, 7)]:
        ref = oracle.solve(g, s, t, d, flags=FLAGS)
        for B in (1, 3, 64):
            r = mos.mos_solve(G, s, t, batch_width=B, pop_order="generation", mem_budget=1 << 28)
            assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, s, t, B)
            check_paths(g, s, t, r.costs, r.paths, d)


def test_routes_and_batches_in_generation_order(mos):
    # a 12-objective time-expanded route, and short ship-grid queries in one batch
    g, s, t = gen.tmplar_route(4, 12, 0)
    G = mos.Graph.from_gen(g)
    lex = mos.mos_solve(G, s, t, n_objectives=12, batch_width=1024)
    gen_ = mos.mos_solve(G, s, t, n_objectives=12, batch_width=1024, pop_order="generation")
    assert np.array_equal(lex.costs, gen_.costs)
    print(f"route 4 d=12: pops lexicographic {lex.stats['pops']}, generation {gen_.stats['pops']}")
    g = gen.ship_grid(256, 256, 3, 0)
    S, T = gen.ship_queries(256, 256, 16, seed=91, dmin=10, dmax=50)
    res = mos.mos_solve_batch(mos.Graph.from_gen(g), S, T, batch_width=512, max_slots=8,
                              pop_order="generation", mem_budget=8 << 30)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q


def test_session_prefix_holds_in_generation_order(mos):
    # the bound of a so-far front is computed from the labels' F1, not from the
    # OPEN key, so the exact prefix holds in any order
    from prefix import compare_prefix

    g, s, t = gen.config1(2)
    ref = oracle.solve(g, s, t, 3, flags=FLAGS)
    sess = mos.Session(mos.Graph.from_gen(g), s, t, batch_width=64, pop_order="generation",
                       mem_budget=1 << 30)
    for _ in range(10):
        sess.step(6)
        r, m = sess.front_so_far()
        compare_prefix(r.costs, m, ref.costs, None)

"""Eager goal front (eager_goal=1): a label accepted at the goal joins the goal
front in the next step's goal step instead of waiting in OPEN until it is
popped.  The front must not change (the oracle decides, bit for bit); the
goal front fills sooner, so fewer labels are expanded and fewer steps run.
Also with the relaxed generation order and the approximate mode, and the
exact prefix of a session still holds."""
import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths
from prefix import compare_prefix

pytestmark = pytest.mark.gpu

FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


@pytest.mark.parametrize("seed", list(range(12)) + [43])
def test_random_multigraphs(mos, seed):
    d = 1 + seed % 4 if seed != 43 else 4
    for g in (gen.random_small(9, 26, d, seed=seed), gen.random_small(9, 20, d, seed=seed)):
        G = mos.Graph.from_gen(g)
        for s, t in [(0, 8), (3, 5), (6, 6), (8, 0)]:
            ref = oracle.solve(g, s, t, d, flags=FLAGS)
            for B in (1, 4, 64):
                r = mos.mos_solve(G, s, t, batch_width=B, eager_goal=True, mem_budget=1 << 28)
                assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, s, t, B)
                check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("B", [256, 32768])
def test_grid_queries(mos, B):
    for seed in (0, 5):
        g, s, t = gen.config1(seed)
        G = mos.Graph.from_gen(g)
        ref = oracle.solve(g, s, t, 3, flags=FLAGS)
        lazy = mos.mos_solve(G, s, t, batch_width=B, costs_only=True, mem_budget=1 << 30)
        eager = mos.mos_solve(G, s, t, batch_width=B, eager_goal=True, mem_budget=1 << 30)
        assert np.array_equal(eager.costs.astype(np.int64), ref.costs), (seed, B)
        check_paths(g, s, t, eager.costs, eager.paths, 3)
        print(f"seed {seed} B {B}: steps {lazy.stats['steps']} -> {eager.stats['steps']}, "
              f"pops {lazy.stats['pops']} -> {eager.stats['pops']}")


def test_routes_orders_and_approximate(mos):
    g, s, t = gen.tmplar_route(4, 12, 0)
    G = mos.Graph.from_gen(g)
    ref = oracle.solve(g, s, t, 12, flags=FLAGS)
    for order in ("lexicographic", "generation"):
        r = mos.mos_solve(G, s, t, n_objectives=12, batch_width=1024, eager_goal=True,
                          pop_order=order)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), order
    apx = mos.mos_solve(G, s, t, n_objectives=12, batch_width=1024, eager_goal=True,
                        epsilon_ppm=20_000)
    assert oracle.first_uncovered(ref.costs, apx.costs.astype(np.int64), 20_000) == -1
    assert oracle.first_dominated(apx.costs) == -1
    # a batch of ship-grid queries
    sg = gen.ship_grid(256, 256, 3, 0)
    S, T = gen.ship_queries(256, 256, 12, seed=17, dmin=10, dmax=50)
    res = mos.mos_solve_batch(mos.Graph.from_gen(sg), S, T, batch_width=512, max_slots=4,
                              eager_goal=True, mem_budget=8 << 30)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK
        ref = oracle.solve(sg, int(S[q]), int(T[q]), 3, flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q


def test_session_prefix_with_eager_goal(mos):
    g, s, t = gen.config1(6)
    ref = oracle.solve(g, s, t, 3, flags=FLAGS)
    sess = mos.Session(mos.Graph.from_gen(g), s, t, batch_width=256, eager_goal=True,
                       mem_budget=1 << 30)
    n = 0
    for _ in range(8):
        sess.step(40)
        r, m = sess.front_so_far()
        n += compare_prefix(r.costs, m, ref.costs, None)
    assert n > 0

"""Seeded generators: same bytes per seed, and the shapes the workloads specify."""
import numpy as np

import gen


def test_config1_shape_and_determinism():
    g, s, t = gen.config1(0)
    assert (g.n, g.n_arcs, g.D, s, t) == (1024, 3968, 3, 0, 1023)
    assert g.cost.min() >= 1 and g.cost.max() <= 10
    assert np.diff(g.row_ptr).max() == 4
    assert g.digest() == gen.config1(0)[0].digest()
    assert g.digest() != gen.config1(1)[0].digest()
    assert gen.overflow_bound_ok(g)


def test_config2_shape():
    g, s, t = gen.config2(0)
    assert (g.n, g.n_arcs, g.D, s, t) == (65536, 521220, 3, 0, 65535)
    assert g.cost.min() >= 100 and g.cost.max() <= 424
    assert np.diff(g.row_ptr).max() == 8


def test_symmetric_arcs_share_costs():
    g, _, _ = gen.config1(3)
    src = g.arc_sources()
    fwd = {(int(a), int(b)): tuple(c) for a, b, c in zip(src, g.col, g.cost)}
    for (a, b), c in fwd.items():
        assert fwd[(b, a)] == c


def test_config3_recipe_counts():
    g, s, t = gen.config3(0)
    assert g.n == 200_000 and g.n_arcs == 1_411_190 and g.D == 4
    assert int(((g.cost == 0).all(1)).sum()) // 2 == 155
    assert np.diff(g.row_ptr).max() == 14
    assert np.linalg.norm(g.coords[s] - g.coords[t]) >= 0.7
    assert gen.overflow_bound_ok(g)


def test_config5_recipe_counts():
    # the served graph's recipe facts for seed 0: 1M points, 8-NN symmetric
    # edges, one component, 3,968 zero-cost edges, 5 objectives
    g, _, comp = gen.config5_graph(0)
    assert g.n == 1_000_000 and g.n_arcs == 9_226_156 and g.D == 5
    assert int(((g.cost == 0).all(1)).sum()) // 2 == 3968
    assert np.diff(g.row_ptr).max() == 18
    assert np.bincount(comp).max() == g.n
    assert gen.overflow_bound_ok(g)
    S, T, D = gen.c5_parity_queries(g, comp, 200, seed=0)
    assert np.all(S != T) and list(D[:6]) == [3, 4, 5, 3, 4, 5]
    assert np.array_equal(np.bincount(D)[3:], [67, 67, 66])


def test_config4_queries():
    g, S, T = gen.config4(0, nq=64)
    rr, cc = np.divmod(np.arange(g.n), 256)
    D = np.abs(rr[S] - rr[T]) + np.abs(cc[S] - cc[T])
    assert D.min() >= 10 and D.max() <= 400
    S2, T2 = gen.config4(0, nq=64)[1:]
    assert np.array_equal(S, S2) and np.array_equal(T, T2)


def test_diamond_chain_structure():
    g, s, t = gen.diamond_chain(4)
    assert (s, t) == (0, 8) and g.n == 13 and g.n_arcs == 16


def test_local_queries_stay_within_radius():
    g, rng, comp = gen.geometric_graph(5000, 8, 5, 1)
    S, T, D = gen.local_queries(g, comp, 200, seed=3, radius=0.05)
    giant = np.bincount(comp).argmax()
    assert np.all(S != T)
    assert np.all(comp[S] == giant) and np.all(comp[T] == giant)
    dist = np.linalg.norm(g.coords[S] - g.coords[T], axis=1)
    assert np.all(dist <= 0.05 + 1e-12)
    assert set(np.unique(D)) <= {3, 4, 5}
    S2, T2, D2 = gen.local_queries(g, comp, 200, seed=3, radius=0.05)
    assert np.array_equal(S, S2) and np.array_equal(T, T2) and np.array_equal(D, D2)


def test_time_expanded_route_structure():
    L, W, T = 6, 3, 4
    g, s, t = gen.time_expanded_route(L, W, 12, seed=3, windows=T)
    assert g.n == L * W * T + 1 and t == g.n - 1 and s == (W // 2) * T
    src = g.arc_sources()
    sink_arcs = g.col == t
    # arcs into the sink: one per window of the destination cell, zero cost
    dest = (L - 1) * W + W // 2
    assert np.array_equal(np.sort(src[sink_arcs]), dest * T + np.arange(T))
    assert not g.cost[sink_arcs].any()
    # other arcs: same or next window, same or next along index, at most one across step
    a, b = src[~sink_arcs], g.col[~sink_arcs]
    (ca, ta), (cb, tb) = np.divmod(a, T), np.divmod(b, T)
    assert np.all((tb == ta) | (tb == ta + 1))
    ia, ja = np.divmod(ca, W)
    ib, jb = np.divmod(cb, W)
    assert np.all((ib - ia >= 0) & (ib - ia <= 1) & (np.abs(jb - ja) <= 1) & (ca != cb))
    c = g.cost[~sink_arcs]
    assert np.all(c[:, 0] > 0) and np.all(c >= 0) and c[:, 11].max() <= 100
    # a fast passage (same window) has the slow one's distance and about twice its fuel
    fast = {(x, y, w): k for k, (x, y, w, w2) in enumerate(zip(ca, cb, ta, tb)) if w2 == w}
    n_pairs = 0
    for k, (x, y, w, w2) in enumerate(zip(ca, cb, ta, tb)):
        if w2 == w + 1:
            f = fast[(x, y, w)]
            assert c[f, 0] == c[k, 0] and abs(int(c[f, 1]) - 2 * int(c[k, 1])) <= 1
            n_pairs += 1
    assert n_pairs == np.count_nonzero(tb == ta + 1) > 0
    assert gen.overflow_bound_ok(g)
    # the first d objectives of the d=12 graph are the d-objective graph
    g4, _, _ = gen.time_expanded_route(L, W, 4, seed=3, windows=T)
    assert np.array_equal(g4.cost, g.cost[:, :4]) and np.array_equal(g4.col, g.col)


def test_tmplar_route_node_counts():
    # node counts of Table 2's five routes: 471, 1610, 461, 201, 778
    for r, n in [(1, 471), (2, 1610), (3, 461), (4, 201), (5, 778)]:
        g, s, t = gen.tmplar_route(r, 3, 0)
        assert abs(g.n - n) <= 0.03 * n

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
    kw.setdefault("mem_budget", 4 << 30)  # a small arena: these instances are small
    r = mos.mos_solve(G, s, t, n_objectives=d or 0, **kw)
    return r


def _fronts(mos, g, pairs, **kw):
    """Several queries on one graph through one batched call (one engine)."""
    G = mos.Graph.from_gen(g)
    kw.setdefault("mem_budget", 4 << 30)
    S = np.array([p[0] for p in pairs], dtype=np.int32)
    T = np.array([p[1] for p in pairs], dtype=np.int32)
    res = mos.mos_solve_batch(G, S, T, **kw)
    assert all(st == mos.MOS_OK for st, _ in res)
    return [r for _, r in res]


@pytest.mark.parametrize("seed", [0, 1])
def test_heuristic_matches_dijkstra(mos, seed):
    g, s, t = gen.config1(seed)
    G = mos.Graph.from_gen(g)
    h = mos.mos_heuristic(G, t)
    ref = oracle.heuristic(g, t)
    ref32 = np.where(ref == oracle.INF, np.iinfo(np.int32).max, ref).astype(np.int32)
    assert np.array_equal(h, ref32)


@pytest.mark.parametrize("which", ["ship256", "road200k", "route1_d12", "road1m"])
def test_heuristic_full_size(mos, which):
    """The heuristic at full size, every node compared: the benchmark's graph
    and goal (256x256 ship grid), the 200k-node road-like query's graph and
    goal, the largest time-expanded route at 12 objectives, and the served
    workload's 1M-node road-like graph with its five stored objectives."""
    if which == "ship256":
        g, s, t = gen.config2(0)
    elif which == "road200k":
        g, s, t = gen.config3(0)
    elif which == "route1_d12":
        g, s, t = gen.tmplar_route(1, 12, seed=0)
    else:
        g, _, _ = gen.config5_graph(0)
        t = 12345
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


@pytest.mark.parametrize("d", [5, 6, 7, 8])
def test_many_objectives(mos, d):
    """The kernels built for 6 and 8 objectives (two int4 words per vector):
    tiny random multigraphs and a 6x6 grid with d objectives."""
    for seed in range(4):
        g = gen.random_small(9, 26, d, seed=100 + 10 * d + seed)
        pairs = [(0, 8), (2, 7)]
        for (s, t), r in zip(pairs, _fronts(mos, g, pairs, batch_width=3)):
            ref = oracle.solve(g, s, t)
            assert np.array_equal(r.costs.astype(np.int64), ref.costs), (d, seed, s, t)
            check_paths(g, s, t, r.costs, r.paths, d)
    g = gen.grid_uniform(6, 6, d, 1, 10, seed=d)
    r = _front(mos, g, 0, g.n - 1, batch_width=64)
    ref = oracle.solve(g, 0, g.n - 1)
    assert np.array_equal(r.costs.astype(np.int64), ref.costs)
    check_paths(g, 0, g.n - 1, r.costs, r.paths, d)


@pytest.mark.parametrize("B", [1, 2, 5, 33])
def test_random_multigraphs(mos, B):
    """Random multigraphs with zero-cost arcs, self-loops and parallel arcs,
    d in 1..4, several start/goal pairs each, at small batch widths."""
    for seed in range(15):
        d = 1 + seed % 4
        g = gen.random_small(11, 34, d, seed=500 + seed)
        pairs = [(0, 10), (4, 4), (7, 2), (1, 9)]
        for (s, t), r in zip(pairs, _fronts(mos, g, pairs, batch_width=B)):
            ref = oracle.solve(g, s, t)
            assert np.array_equal(r.costs.astype(np.int64), ref.costs), (B, seed, s, t)
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


@pytest.mark.parametrize("seed", [0, 3, 5, 8])
def test_batch_of_one_pops_like_the_oracle(mos, seed):
    """With B = 1 each step pops the single lexicographically smallest live
    label, so the GPU processes exactly the labels sequential NAMOA* processes
    (weak goal-front tests, PruneOPEN applied when a label is popped)."""
    g = gen.grid_uniform(10, 10, 3, 1, 10, seed=seed)
    r = _front(mos, g, 0, g.n - 1, batch_width=1, heuristic_radius=-1)
    ref = oracle.solve(g, 0, g.n - 1, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
    assert np.array_equal(r.costs.astype(np.int64), ref.costs)
    assert r.stats["pops"] == ref.stats["pops"]
    assert r.stats["steps"] >= r.stats["pops"]


def test_repeatable_paths(mos):
    g, s, t = gen.config1(4)
    a = _front(mos, g, s, t, batch_width=512)
    b = _front(mos, g, s, t, batch_width=512)
    assert np.array_equal(a.costs, b.costs)
    assert all(np.array_equal(x, y) for x, y in zip(a.paths, b.paths))


@pytest.mark.parametrize("size", [48, 96])
def test_ship_grid_front(mos, size):
    g, s, t = gen.config2(0, size=size)
    r = _front(mos, g, s, t, batch_width=1024)
    ref = oracle.solve(g, s, t, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
    assert np.array_equal(r.costs.astype(np.int64), ref.costs)
    check_paths(g, s, t, r.costs, r.paths, 3)


@pytest.mark.parametrize("B", [4096, 32768])
def test_widest_batches(mos, B):
    """Batches up to the largest width (16 popped labels per thread of the
    per-query workgroup) on the 32x32 grid and the 96x96 ship grid."""
    for g, s, t in (gen.config1(0), gen.config2(0, size=96)):
        r = _front(mos, g, s, t, batch_width=B)
        ref = oracle.solve(g, s, t, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs)
        check_paths(g, s, t, r.costs, r.paths, 3)


@pytest.mark.parametrize("radius", [-1, 1, 2])
def test_front_does_not_depend_on_heuristic_radius(mos, radius):
    """Exact heuristic (-1) or a reverse search cut at radius x h(start) with the
    lower bound beyond it: same front, only the work differs."""
    g64, _, _ = gen.config2(0, size=64)
    g1, s1, t1 = gen.config1(3)
    # interior queries: with radius 1 most of the grid lies beyond the cut
    cases = ((g1, s1, t1), (g64, 0, 64 * 64 - 1), (g1, 10 * 32 + 10, 16 * 32 + 16),
             (g1, 12 * 32 + 8, 18 * 32 + 20))
    for g, s, t in cases:
        r = _front(mos, g, s, t, batch_width=512, heuristic_radius=radius)
        ref = oracle.solve(g, s, t, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs)
        check_paths(g, s, t, r.costs, r.paths, 3)


def test_diamond_chain_large_front(mos):
    g, s, t = gen.diamond_chain(12)
    r = _front(mos, g, s, t, batch_width=256)
    W = 2 ** 12 - 1
    expect = np.array([[x, W - x] for x in range(2 ** 12)], dtype=np.int64)
    assert np.array_equal(r.costs.astype(np.int64), expect)
    check_paths(g, s, t, r.costs, r.paths, 2)


def test_unreachable_and_trivial(mos):
    g2 = gen.from_arcs(4, [0, 1, 2], [1, 0, 3], np.ones((3, 2), dtype=np.int64))
    G = mos.Graph.from_gen(g2)
    assert mos.mos_solve(G, 0, 3).costs.shape == (0, 2)
    r = mos.mos_solve(G, 2, 2)
    assert r.costs.tolist() == [[0, 0]] and len(r.paths[0]) == 0


def test_invalid_arguments_rejected(mos):
    """Out-of-range options and queries fail with MOS_E_INVALID_ARG before any
    search runs, and the library keeps working afterwards."""
    g = gen.random_small(9, 26, 2, seed=1)
    G = mos.Graph.from_gen(g)
    bad = [dict(batch_width=32769), dict(batch_width=-1), dict(steps_per_poll=1025),
           dict(label_limit=-1), dict(n_objectives=3)]
    for kw in bad:
        with pytest.raises(mos.MosError) as e:
            mos.mos_solve(G, 0, 8, **kw)
        assert e.value.status == mos.MOS_E_INVALID_ARG, kw
    for s, t in [(-1, 8), (0, g.n)]:
        with pytest.raises(mos.MosError) as e:
            mos.mos_solve(G, s, t)
        assert e.value.status == mos.MOS_E_INVALID_ARG, (s, t)
    # the widest batch is accepted, and the front is still the oracle's
    r = mos.mos_solve(G, 0, 8, batch_width=32768)
    assert np.array_equal(r.costs.astype(np.int64), oracle.solve(g, 0, 8).costs)


def test_session_matches_solve(mos):
    g, s, t = gen.config1(1)
    G = mos.Graph.from_gen(g)
    ref = mos.mos_solve(G, s, t, batch_width=512)
    sess = mos.Session(G, s, t, batch_width=512, profile_kernels=True)
    done = sess.step(5)
    st5 = sess.stats()
    assert not done and st5["steps"] == 5
    r = sess.result()
    assert np.array_equal(r.costs, ref.costs)
    assert all(np.array_equal(x, y) for x, y in zip(r.paths, ref.paths))
    kt = sess.kernel_times()
    assert kt["k_group_process"][1] >= r.stats["steps"]  # steps after the end are no-ops
    assert sum(v[0] for v in kt.values()) > 0
    sess.close()

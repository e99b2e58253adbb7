"""One workgroup per query (persistent_query=1): each resident query runs its
label steps inside one workgroup of its own, many steps per launch, with
workgroup barriers between the phases (the batched extraction of Section 5
without a launch per phase).  The front must equal the oracle's bit for bit
(Section 3's answer: the set of non-dominated cost vectors), every witness path
must re-sum to its costs, and a query's output (paths included) must not
depend on the other queries of the batch nor on the run."""
import time

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


def _same_output(a, b):
    return np.array_equal(a.costs, b.costs) and all(
        np.array_equal(x, y) for x, y in zip(a.paths, b.paths))


@pytest.mark.parametrize("seed", range(12))
def test_random_multigraphs(mos, seed):
    """Small random multigraphs (self-loops, parallel arcs, zero costs) at
    d = 1..4.  Width 1 makes most steps end in ties of the smallest F1 wider
    than the batch: those queries leave for the multi-kernel step and must
    still come out exact."""
    d = 1 + seed % 4
    for g in (gen.random_small(9, 26, d, seed=seed), gen.random_small(9, 20, d, seed=seed)):
        G = mos.Graph.from_gen(g)
        for s, t in [(0, 8), (3, 5), (6, 6), (8, 0)]:
            ref = oracle.solve(g, s, t, d, flags=FLAGS)
            for B in (1, 4, 64, 1024):
                r = mos.mos_solve(G, s, t, batch_width=B, persistent_query=True,
                                  mem_budget=1 << 28)
                assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, s, t, B)
                check_paths(g, s, t, r.costs, r.paths, d)


def test_unreachable_goal_and_start_is_goal(mos):
    g = gen.random_small(12, 14, 3, seed=5, self_loops=True)
    G = mos.Graph.from_gen(g)
    for s in range(g.n):
        for t in range(g.n):
            ref = oracle.solve(g, s, t, 3, flags=FLAGS)
            r = mos.mos_solve(G, s, t, batch_width=64, persistent_query=True, mem_budget=1 << 28)
            assert np.array_equal(r.costs.astype(np.int64), ref.costs), (s, t)
            check_paths(g, s, t, r.costs, r.paths, 3)


@pytest.mark.parametrize("B", [64, 256, 1024])
def test_grid_queries(mos, B):
    """The 32x32 grid recipe, corner to corner (fronts of hundreds of vectors)."""
    for seed in (0, 5, 9):
        g, s, t = gen.config1(seed)
        G = mos.Graph.from_gen(g)
        ref = oracle.solve(g, s, t, 3, flags=FLAGS)
        r = mos.mos_solve(G, s, t, batch_width=B, persistent_query=True, mem_budget=1 << 30)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, B)
        check_paths(g, s, t, r.costs, r.paths, 3)
        again = mos.mos_solve(G, s, t, batch_width=B, persistent_query=True, mem_budget=1 << 30)
        assert _same_output(r, again), (seed, B)


def test_ship_batch_alone_and_mixed_objectives(mos):
    """Short queries of the batched workload's recipe on the 256x256 ship grid
    (Manhattan distance 10..60), in one batch: oracle fronts, the same output
    alone, and objective counts mixed within the batch."""
    g = gen.ship_grid(256, 256, 3, 0)
    G = mos.Graph.from_gen(g)
    S, T = gen.ship_queries(256, 256, 40, seed=77, dmin=10, dmax=60)
    res = mos.mos_solve_batch(G, S, T, batch_width=1024, max_slots=16, persistent_query=True,
                              mem_budget=8 << 30)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK, q
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q
        check_paths(g, int(S[q]), int(T[q]), r.costs, r.paths, 3)
    for q in range(0, 40, 9):
        alone = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=1024, persistent_query=True,
                              mem_budget=8 << 30)
        assert _same_output(alone, res[q][1]), q
    D = np.array([1 + q % 3 for q in range(12)], dtype=np.int32)
    mixed = mos.mos_solve_batch(G, S[:12], T[:12], n_objectives=D, batch_width=512,
                                max_slots=8, persistent_query=True, mem_budget=8 << 30)
    for q, (st, r) in enumerate(mixed):
        assert st == mos.MOS_OK, q
        ref = oracle.solve(g, int(S[q]), int(T[q]), int(D[q]), flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q


def test_routes_two_and_five(mos):
    """Two stored time-expanded route fronts at Table 2's objective counts."""
    import glob
    import importlib.util
    import os

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "make_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    files = {int(os.path.basename(f)[1]): f
             for f in glob.glob(os.path.join(here, "routes", "r*.txt.gz"))}
    for r in (2, 5):
        h, costs = m.read_front(files[r])
        d = gen.ROUTE_MAX_OBJECTIVES[r]
        g, s, t = gen.tmplar_route(r, 12, 0)
        assert h["graph_sha256_16"] == g.digest()
        res = mos.mos_solve(mos.Graph.from_gen(g), s, t, n_objectives=d, batch_width=1024,
                            persistent_query=True, mem_budget=16 << 30)
        assert np.array_equal(res.costs.astype(np.int64), costs), r
        check_paths(g, s, t, res.costs, res.paths, d)


def test_server_and_readmission(mos):
    """The request loop in this mode on a 20k-node road-like graph (d in
    {3, 4, 5}), against the oracle; then a memory budget the first
    reservation outgrows, so that queries are re-admitted."""
    from scipy.spatial import cKDTree

    g, rng, comp = gen.geometric_graph(20000, 8, 5, 0)
    tree = cKDTree(g.coords)
    r = np.random.default_rng(11)
    giant = np.bincount(comp).argmax()
    qs = []
    while len(qs) < 24:
        s = int(r.integers(0, g.n))
        if comp[s] != giant:
            continue
        near = tree.query_ball_point(g.coords[s], 0.12)
        qs.append((s, int(near[r.integers(0, len(near))]), int(r.integers(3, 6))))
    G = mos.Graph.from_gen(g)
    srv = mos.Server(G, mem_budget=8 << 30, max_slots=8, persistent_query=True)
    try:
        tickets = []
        for i, (s, t, d) in enumerate(qs):
            tickets.append(srv.submit(s, t, d))
            if i % 8 == 7:
                time.sleep(0.01)
        out = [srv.wait(tk, timeout_ms=120000) for tk in tickets]
    finally:
        srv.close()
    for (s, t, d), o in zip(qs, out):
        assert o is not None and o[0] == mos.MOS_OK
        ref = oracle.solve(g, s, t, d, flags=FLAGS)
        assert np.array_equal(o[1].costs.astype(np.int64), ref.costs)
        check_paths(g, s, t, o[1].costs, o[1].paths, d)
    g1, _, _ = gen.config1(2)
    G1 = mos.Graph.from_gen(g1)
    S = np.zeros(4, dtype=np.int32)
    T = np.array([1023, 500, 700, 1000], dtype=np.int32)
    srv = mos.Server(G1, mem_budget=96 << 20, max_slots=4, persistent_query=True)
    try:
        got = [srv.wait(srv.submit(int(S[q]), int(T[q]), 3)) for q in range(4)]
        c = srv.counters()
    finally:
        srv.close()
    assert c["readmissions"] > 0
    for q, (st, res) in enumerate(got):
        ref = oracle.solve(g1, int(S[q]), int(T[q]), 3, flags=FLAGS)
        assert st == mos.MOS_OK and np.array_equal(res.costs.astype(np.int64), ref.costs), q


def test_ignored_with_step_budget(mos):
    """With a step budget the query runs the multi-kernel step: its prefix
    is that mode's, exact below the reported bound."""
    from prefix import compare_prefix

    g = gen.ship_grid(256, 256, 3, 0)
    G = mos.Graph.from_gen(g)
    S, T = gen.ship_queries(256, 256, 3, seed=404, dmin=30, dmax=75)
    for q in range(3):
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=FLAGS)
        a = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=256, step_budget=16,
                          steps_per_poll=8, persistent_query=True, mem_budget=8 << 30)
        b = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=256, step_budget=16,
                          steps_per_poll=8, mem_budget=8 << 30)
        assert _same_output(a, b), q
        if not a.complete:
            assert compare_prefix(a.costs, a.stats["open_min_f1"], ref.costs, None) == a.costs.shape[0]

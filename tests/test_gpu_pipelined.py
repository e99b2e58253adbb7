"""Pipelined steps (pipelined=1): the goal-front filter of a step's new labels
runs at the start of the next step, beside that step's pop, on a second
stream (the extraction of the next batch overlaps the last stage of the
current one, Section 5.1's current and next bags).  The front must not change
(the oracle decides, bit for bit, at batch widths 1 to 32768, on the routes
at Table 2's objective counts, in batches and in the server); a step-limited
prefix stays exact; profiled steps run the same kernels in order on one
stream."""
import glob
import importlib.util
import os

import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths
from prefix import compare_prefix

pytestmark = pytest.mark.gpu

FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def _read_front():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m.read_front


@pytest.mark.parametrize("seed", range(12))
def test_random_multigraphs(mos, seed):
    d = 1 + seed % 4
    for g in (gen.random_small(9, 26, d, seed=seed), gen.random_small(9, 20, d, seed=seed)):
        G = mos.Graph.from_gen(g)
        for s, t in [(0, 8), (3, 5), (6, 6), (8, 0)]:
            ref = oracle.solve(g, s, t, d, flags=FLAGS)
            for B in (1, 4, 64, 1024):
                r = mos.mos_solve(G, s, t, batch_width=B, pipelined=True, mem_budget=1 << 28)
                assert np.array_equal(r.costs.astype(np.int64), ref.costs), (seed, s, t, B)
                check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("B", [64, 1024, 32768])
def test_grid_queries(mos, B):
    for seed in (0, 5):
        g, s, t = gen.config1(seed)
        G = mos.Graph.from_gen(g)
        ref = oracle.solve(g, s, t, 3, flags=FLAGS)
        sync = mos.mos_solve(G, s, t, batch_width=B, costs_only=True, mem_budget=1 << 30)
        pipe = mos.mos_solve(G, s, t, batch_width=B, pipelined=True, mem_budget=1 << 30)
        assert np.array_equal(pipe.costs.astype(np.int64), ref.costs), (seed, B)
        check_paths(g, s, t, pipe.costs, pipe.paths, 3)
        print(f"seed {seed} B {B}: steps {sync.stats['steps']} -> {pipe.stats['steps']}, "
              f"pops {sync.stats['pops']} -> {pipe.stats['pops']}")


def test_routes(mos):
    """The five stored route fronts (up to 12 objectives, up to 79,250 vectors)."""
    read_front = _read_front()
    files = sorted(glob.glob(os.path.join(HERE, "routes", "r*.txt.gz")))
    assert len(files) == 5
    for f in files:
        h, costs = read_front(f)
        r = int(os.path.basename(f)[1])
        d = gen.ROUTE_MAX_OBJECTIVES[r]
        g, s, t = gen.tmplar_route(r, 12, 0)
        assert h["graph_sha256_16"] == g.digest()
        res = mos.mos_solve(mos.Graph.from_gen(g), s, t, n_objectives=d, batch_width=4096,
                            pipelined=True, mem_budget=16 << 30)
        assert np.array_equal(res.costs.astype(np.int64), costs), r
        check_paths(g, s, t, res.costs, res.paths, d)


def test_batch_alone_and_mix_and_server(mos):
    sg = gen.ship_grid(256, 256, 3, 0)
    G = mos.Graph.from_gen(sg)
    S, T = gen.ship_queries(256, 256, 12, seed=23, dmin=10, dmax=50)
    res = mos.mos_solve_batch(G, S, T, batch_width=512, max_slots=4, pipelined=True,
                              mem_budget=8 << 30)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK
        ref = oracle.solve(sg, int(S[q]), int(T[q]), 3, flags=FLAGS)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q
        alone = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=512, pipelined=True,
                              mem_budget=8 << 30)
        assert np.array_equal(alone.costs, r.costs), q
        check_paths(sg, int(S[q]), int(T[q]), r.costs, r.paths, 3)
    srv = mos.Server(G, mem_budget=8 << 30, max_slots=4, batch_width=512, pipelined=True)
    try:
        tickets = [srv.submit(int(S[q]), int(T[q])) for q in range(6)]
        for q, tk in enumerate(tickets):
            st, r = srv.wait(tk)
            assert st == mos.MOS_OK and np.array_equal(r.costs, res[q][1].costs), q
    finally:
        srv.close()


def test_step_budget_prefix_and_eager(mos):
    g = gen.ship_grid(256, 256, 3, 0)
    G = mos.Graph.from_gen(g)
    S, T = gen.ship_queries(256, 256, 6, seed=404, dmin=30, dmax=75)
    for q in range(6):
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=FLAGS)
        r = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=256, step_budget=16,
                          steps_per_poll=8, pipelined=True, mem_budget=8 << 30)
        if r.complete:
            assert np.array_equal(r.costs.astype(np.int64), ref.costs), q
        else:
            n = compare_prefix(r.costs, r.stats["open_min_f1"], ref.costs, None)
            assert n == r.costs.shape[0], q
        e = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=256, pipelined=True,
                          eager_goal=True, mem_budget=8 << 30)
        assert np.array_equal(e.costs.astype(np.int64), ref.costs), q


def test_session_prefix_and_profiled_steps(mos):
    g, s, t = gen.config1(6)
    ref = oracle.solve(g, s, t, 3, flags=FLAGS)
    sess = mos.Session(mos.Graph.from_gen(g), s, t, batch_width=256, pipelined=True,
                       mem_budget=1 << 30)
    n = 0
    for _ in range(8):
        sess.step(40)
        r, m = sess.front_so_far()
        n += compare_prefix(r.costs, m, ref.costs, None)
    assert n > 0
    # profile mode: the same kernels in order on one stream, every kernel timed
    prof = mos.Session(mos.Graph.from_gen(g), s, t, batch_width=256, pipelined=True,
                       profile_kernels=True, mem_budget=1 << 30)
    while not prof.step(16):
        pass
    times = prof.kernel_times()
    assert times["k_pfilter"][1] > 0 and times["k_group_pairs"][1] > 0
    out = prof.result()
    assert np.array_equal(out.costs.astype(np.int64), ref.costs)

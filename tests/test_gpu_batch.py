"""Batched form: many queries resident at once, admitted into slots as they free up.

Every query's front must equal the oracle's, and a query's output (paths
included) must not depend on the other queries of the batch.
"""
import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


@pytest.fixture(scope="module")
def ship():
    """The seed-0 256x256 ship grid and short-range queries drawn with the
    batched workload's recipe (Manhattan distance uniform in [10, 60])."""
    g = gen.ship_grid(256, 256, 3, 0)
    S, T = gen.ship_queries(256, 256, 40, seed=77, dmin=10, dmax=60)
    return g, S, T


def test_batch_matches_oracle_and_alone(mos, ship):
    g, S, T = ship
    G = mos.Graph.from_gen(g)
    res = mos.mos_solve_batch(G, S, T, batch_width=256, max_slots=16)
    assert len(res) == len(S)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK, q
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q
        check_paths(g, int(S[q]), int(T[q]), r.costs, r.paths, 3)
    # alone == in the mix, paths included (same batch width)
    for q in range(0, len(S), 5):
        alone = mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=256)
        assert np.array_equal(alone.costs, res[q][1].costs)
        assert all(np.array_equal(a, b) for a, b in zip(alone.paths, res[q][1].paths)), q


def test_batch_mixed_objectives(mos, ship):
    g, S, T = ship
    G = mos.Graph.from_gen(g)
    nobj = np.array([1 + q % 3 for q in range(12)], dtype=np.int32)
    res = mos.mos_solve_batch(G, S[:12], T[:12], n_objectives=nobj, batch_width=128, max_slots=5)
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK
        ref = oracle.solve(g, int(S[q]), int(T[q]), int(nobj[q]),
                           flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), q


def test_batch_label_limit_is_per_query(mos):
    """A query that outgrows label_limit fails cleanly; the others are exact."""
    g, s, t = gen.config1(0)
    small = gen.grid_uniform(6, 6, 3, 1, 10, seed=2)
    G = mos.Graph.from_gen(g)
    S = np.array([0, 0, 5], dtype=np.int32)
    T = np.array([1023, 33, 38], dtype=np.int32)
    res = mos.mos_solve_batch(G, S, T, batch_width=256, label_limit=20000, max_slots=3)
    assert res[0][0] == mos.MOS_E_LABEL_LIMIT and res[0][1] is None
    for q in (1, 2):
        assert res[q][0] == mos.MOS_OK
        ref = oracle.solve(g, int(S[q]), int(T[q]), 3)
        assert np.array_equal(res[q][1].costs.astype(np.int64), ref.costs)
    del small


def test_small_budget_readmits(mos):
    """With a memory budget that the first reservation outgrows, queries are
    re-admitted with a larger reservation and still come out exact."""
    g, s, t = gen.config1(2)
    G = mos.Graph.from_gen(g)
    S = np.zeros(4, dtype=np.int32)
    T = np.array([1023, 500, 700, 1000], dtype=np.int32)
    res = mos.mos_solve_batch(G, S, T, batch_width=256, max_slots=4, mem_budget=256 << 20)
    refs = [oracle.solve(g, int(S[q]), int(T[q]), 3).costs for q in range(4)]
    for q, (st, r) in enumerate(res):
        assert st == mos.MOS_OK, q
        assert np.array_equal(r.costs.astype(np.int64), refs[q]), q
    # the same through the request loop, whose counters show the re-admissions
    srv = mos.Server(G, mem_budget=96 << 20, max_slots=4)
    tickets = [srv.submit(int(S[q]), int(T[q]), 3) for q in range(4)]
    got = [srv.wait(tk) for tk in tickets]
    c = srv.counters()
    srv.close()
    assert c["readmissions"] > 0
    for q, (st, r) in enumerate(got):
        assert st == mos.MOS_OK and np.array_equal(r.costs.astype(np.int64), refs[q]), q


def test_autotuned_batch_width(mos):
    """The autotuner returns one of its widths, and the fronts at that width
    equal the oracle's."""
    from paper_2411_16667_amd.autotune import tune_batch_width

    g = gen.grid_uniform(12, 12, 3, 1, 10, seed=21)
    G = mos.Graph.from_gen(g)
    rng = np.random.default_rng(5)
    S = rng.integers(0, g.n, 10).astype(np.int32)
    T = rng.integers(0, g.n, 10).astype(np.int32)
    r = tune_batch_width(G, S, T, widths=(4, 64, 512), sample=6, mem_budget=2 << 30)
    assert r["batch_width"] in (4, 64, 512) and set(r["seconds"]) == {4, 64, 512}
    res = mos.mos_solve_batch(G, S, T, batch_width=r["batch_width"], mem_budget=2 << 30)
    for (st, x), s, t in zip(res, S, T):
        assert st == mos.MOS_OK
        assert np.array_equal(x.costs.astype(np.int64), oracle.solve(g, int(s), int(t)).costs)

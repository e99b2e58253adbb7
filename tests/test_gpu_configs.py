"""The batched and served configurations as generated, against the oracle.

* The 512-query batch on the 256x256 ship grid (Manhattan distances
  U{10..400}) in ONE mos_solve_batch call with a step budget: every query
  returns either its complete front or, at the budget, the exact part of its
  front below its bound.  The oracle ran every query for a bounded time
  (tests/golden/c4batch.txt.gz: complete fronts, or exact prefixes below the
  F of its smallest open label).  On the common range the two must agree
  entry for entry; complete GPU fronts must also meet the necessary
  conditions (ideal point, all lexicographic extremes, supported points).
* 200 uniformly random pairs on the 1M-node road-like graph, a third each at
  3, 4 and 5 objectives, through the request loop (mos_server_*), compared
  the same way with tests/golden/c5_subset.txt.gz; a sample is solved again
  alone and must come back identical (costs and paths).
"""
import importlib.util
import os

import numpy as np
import pytest

import gen
from helpers import check_paths
from prefix import compare_prefix, necessary_conditions

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def _bound(e):
    return e.get("bound") if e["complete"] == "0" else None


def test_c4_batch_of_512_as_generated(mos):
    hdr, entries = _golden().read_front_set(os.path.join(HERE, "c4batch.txt.gz"))
    g, S, T = gen.config4(0)
    assert hdr["graph_sha256_16"] == g.digest() and len(entries) == len(S) == 512
    for q, (e, _) in enumerate(entries):
        assert (int(e["start"]), int(e["goal"])) == (int(S[q]), int(T[q]))
    G = mos.Graph.from_gen(g)
    res = mos.mos_solve_batch(G, S, T, batch_width=1024, max_slots=256, step_budget=256,
                              steps_per_poll=16)
    assert len(res) == 512
    done = compared = 0
    for q, ((st, r), (e, rows)) in enumerate(zip(res, entries)):
        assert st in (mos.MOS_OK, mos.MOS_E_STEP_LIMIT), (q, st)
        gb = None if st == mos.MOS_OK else r.stats["open_min_f1"]
        compared += compare_prefix(r.costs, gb, rows, _bound(e))
        s, t = int(S[q]), int(T[q])
        if st == mos.MOS_OK:
            done += 1
            if e["complete"] == "1":
                assert np.array_equal(r.costs.astype(np.int64), rows), q
            if r.costs.shape[0] <= 20000:
                necessary_conditions(g, s, t, 3, r.costs, n_weights=3, seed=q)
        if q % 16 == 0 and r.costs.shape[0]:
            idx = np.linspace(0, r.costs.shape[0] - 1, min(32, r.costs.shape[0])).astype(int)
            check_paths(g, s, t, r.costs[idx], [r.paths[i] for i in idx], 3)
    print(f"c4: {done} of 512 complete within 256 steps, {compared} entries compared")
    assert done >= 80 and compared >= 50_000


def test_c5_served_random_pairs(mos):
    hdr, entries = _golden().read_front_set(os.path.join(HERE, "c5_subset.txt.gz"))
    g, _, comp = gen.config5_graph(0)
    S, T, D = gen.c5_parity_queries(g, comp, 200, seed=0)
    assert hdr["graph_sha256_16"] == g.digest() and len(entries) == 200
    G = mos.Graph.from_gen(g)
    opts = dict(batch_width=1024, step_budget=64, steps_per_poll=16)
    srv = mos.Server(G, max_slots=64, **opts)
    tickets = [srv.submit(int(S[q]), int(T[q]), int(D[q])) for q in range(200)]
    got = [srv.wait(tk) for tk in tickets]
    srv.close()
    compared = 0
    for q, ((st, r), (e, rows)) in enumerate(zip(got, entries)):
        assert (int(e["start"]), int(e["goal"]), int(e["d"])) == (int(S[q]), int(T[q]), int(D[q]))
        assert st in (mos.MOS_OK, mos.MOS_E_STEP_LIMIT), (q, st)
        gb = None if st == mos.MOS_OK else r.stats["open_min_f1"]
        compared += compare_prefix(r.costs, gb, rows, _bound(e))
    # alone against the mix: the same costs and the same witness paths
    for q in (0, 1, 2, 97, 198):
        alone = mos.mos_solve(G, int(S[q]), int(T[q]), n_objectives=int(D[q]), **opts)
        st, r = got[q]
        assert np.array_equal(alone.costs, r.costs), q
        assert all(np.array_equal(a, b) for a, b in zip(alone.paths, r.paths)), q
        check_paths(g, int(S[q]), int(T[q]), r.costs[:50], r.paths[:50], int(D[q]))
    print(f"c5: {compared} entries compared over 200 queries")
    assert compared >= 1000

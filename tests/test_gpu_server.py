"""Served form: continuous batching over a request queue.

Requests submitted while others run share the device; each result must be the
oracle's front, and the same as the query solved alone (paths included).
"""
import time

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
def road():
    """A 20k-node 8-NN geometric graph with 5 objectives; queries with d in
    {3, 4, 5} and goals within a bounded radius of the start."""
    from scipy.spatial import cKDTree

    g, rng, comp = gen.geometric_graph(20000, 8, 5, 0)
    tree = cKDTree(g.coords)
    r = np.random.default_rng(11)
    giant = np.bincount(comp).argmax()
    qs = []
    while len(qs) < 48:
        s = int(r.integers(0, g.n))
        if comp[s] != giant:
            continue
        near = tree.query_ball_point(g.coords[s], 0.12)
        t = int(near[r.integers(0, len(near))])
        qs.append((s, t, int(r.integers(3, 6))))
    return g, qs


def test_server_matches_oracle_and_alone(mos, road):
    g, qs = road
    G = mos.Graph.from_gen(g)
    srv = mos.Server(G, mem_budget=8 << 30, max_slots=8)
    tickets = []
    for i, (s, t, d) in enumerate(qs):
        tickets.append(srv.submit(s, t, d))
        if i % 8 == 7:
            time.sleep(0.01)  # arrivals while earlier requests are on the device
    out = [srv.wait(tk, timeout_ms=120000) for tk in tickets]
    c = srv.counters()
    assert c["submitted"] == len(qs) and c["finished"] == len(qs)
    for (s, t, d), o in zip(qs, out):
        assert o is not None and o[0] == mos.MOS_OK
        r = o[1]
        ref = oracle.solve(g, s, t, d, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
        assert np.array_equal(r.costs.astype(np.int64), ref.costs)
        check_paths(g, s, t, r.costs, r.paths, d)
    # the server runs B = 256: a query alone gives the same output
    for (s, t, d), o in list(zip(qs, out))[::7]:
        alone = mos.mos_solve(G, s, t, n_objectives=d, batch_width=256)
        assert np.array_equal(alone.costs, o[1].costs)
        assert all(np.array_equal(a, b) for a, b in zip(alone.paths, o[1].paths))
    srv.close()


def test_server_cancel_and_poll(mos, road):
    g, qs = road
    G = mos.Graph.from_gen(g)
    srv = mos.Server(G, mem_budget=4 << 30, max_slots=2)
    tks = [srv.submit(s, t, d) for (s, t, d) in qs[:10]]
    srv.cancel(tks[-1])
    got = {}
    deadline = time.time() + 60
    while len(got) < len(tks) and time.time() < deadline:
        for tk in tks:
            if tk in got:
                continue
            o = srv.poll(tk)
            if o is not None:
                got[tk] = o
        time.sleep(0.002)
    assert len(got) == len(tks)
    assert got[tks[-1]][0] in (mos.MOS_E_CANCELLED, mos.MOS_OK)
    for tk, (s, t, d) in zip(tks[:-1], qs[:9]):
        assert got[tk][0] == mos.MOS_OK
        ref = oracle.solve(g, s, t, d)
        assert np.array_equal(got[tk][1].costs.astype(np.int64), ref.costs)
    with pytest.raises(mos.MosError):
        srv.poll(tks[0])  # a ticket is collected once
    srv.close()


def test_loop_failure_reports_every_query():
    """A failure of the request loop, forced from the host by a test hook that
    throws before a given tick (no device fault), ends every query not yet
    reported -- finished that tick, resident, queued or still in the inbox --
    with the error, so that a wait without a time limit returns; a submit
    afterwards fails with the same status.  Run in a child process with a time
    limit, so that a regression (a wait that never returns) fails the test
    instead of hanging the run."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r"""
import gen
import paper_2411_16667_amd as mos
g, s, t = gen.config1(0)
srv = mos.Server(mos.Graph.from_gen(g), max_slots=2, batch_width=64)
tickets = [srv.submit(a, 1023, 3) for a in range(16)]
print("STATUSES", " ".join(str(srv.wait(tk)[0]) for tk in tickets), flush=True)
try:
    srv.submit(0, 1023, 3)
    print("SUBMIT ok")
except mos.MosError as e:
    print("SUBMIT", e.status)
srv.close()
"""
    env = dict(os.environ, MOS_SERVER_FAIL_AT_TICK="3", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = dict(line.split(" ", 1) for line in r.stdout.splitlines() if " " in line)
    import paper_2411_16667_amd as mos

    sts = [int(x) for x in lines["STATUSES"].split()]
    assert len(sts) == 16
    assert set(sts) <= {mos.MOS_OK, mos.MOS_E_DEVICE} and mos.MOS_E_DEVICE in sts, sts
    assert lines["SUBMIT"] == str(mos.MOS_E_DEVICE)

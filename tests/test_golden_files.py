"""The stored oracle fronts under tests/golden/ are what the committed script
and oracle produce today.

For every stored file: the graph regenerated from the seeded generators has
the digest the file records, the start and goal agree, and the costs are a
lexicographically ascending antichain of the recorded size (for fronts above
4000 entries, 2000 seeded rows are checked against the whole front).  The
files whose oracle search took under a second are recomputed with the
oracle, as the script computes them, and must match exactly; so a change to
the generators or the oracle that would make the stored values stale fails
here on the CPU.
"""
import glob
import os

import numpy as np
import pytest

import gen
import oracle
from helpers import is_antichain, sort_lex

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN


def _read_front():
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m.read_front


def _workload(h):
    """Regenerate (graph, start, goal, d) for a stored header."""
    name = h["workload"]
    d = int(h["d"])
    if name.startswith("c1_s"):
        g, s, t = gen.config1(int(name[4:]))
    elif name.startswith("c4mid_q"):
        g = _ship256()
        s, t = int(h["start"]), int(h["goal"])
        S, T = gen.ship_queries(256, 256, 20, seed=99, dmin=60, dmax=120)
        q = int(name[7:])
        assert (int(S[q]), int(T[q])) == (s, t)
    elif name.startswith("route"):
        r = int(name[5:name.index("_")])
        g, s, t = gen.tmplar_route(r, 12, 0)
    else:
        raise AssertionError("unknown stored workload " + name)
    return g, s, t, d


_cache = {}


def _ship256():
    if "ship" not in _cache:
        _cache["ship"] = gen.ship_grid(256, 256, 3, 0)
    return _cache["ship"]


FILES = sorted(glob.glob(os.path.join(HERE, "*", "*.txt.gz")))


def test_stored_files_present():
    names = {os.path.basename(os.path.dirname(f)) for f in FILES}
    assert {"c1", "c4mid", "routes"} <= names
    assert len(glob.glob(os.path.join(HERE, "c1", "*.txt.gz"))) == 32


@pytest.mark.parametrize("path", FILES, ids=[os.path.relpath(f, HERE) for f in FILES])
def test_stored_front(path):
    h, costs = _read_front()(path)
    g, s, t, d = _workload(h)
    assert h["graph_sha256_16"] == g.digest()
    assert (int(h["start"]), int(h["goal"])) == (s, t)
    assert costs.shape == (int(h["front"]), d)
    assert np.array_equal(costs, sort_lex(costs))
    if costs.shape[0] <= 4000:
        assert is_antichain(costs)
    else:  # large fronts: a seeded sample of rows against the whole front
        rows = np.random.default_rng(0).choice(costs.shape[0], 2000, replace=False)
        for i in rows:
            le = np.all(costs <= costs[i], axis=1)
            le[i] = False
            assert not le.any(), i
    if float(h["search_seconds"]) < 1.0:
        r = oracle.solve(g, s, t, d, flags=int(h["oracle_flags"]))
        assert r.status == "ok"
        assert np.array_equal(r.costs, costs)

"""Approximate fronts on the GPU (epsilon_ppm > 0; the paper's Sections 2 and 8
name epsilon-dominance as the way to trade exactness for work).

The approximate front is not unique (it depends on the order goal labels
arrive in), so it is checked by what must hold of any valid answer, against
the exact front from the oracle: every exact vector y has an entry a with
a <= (1 + eps) y (the oracle's cover check), the entries are mutually
non-dominated, each is the re-summed cost of its own witness path, and there
are no more of them than exact vectors.  epsilon 0 must give the exact front.
"""
import glob
import importlib.util
import os

import numpy as np
import pytest

import gen
import oracle
from helpers import check_paths

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def _valid(g, s, t, d, exact, r, ppm):
    got = r.costs.astype(np.int64)
    assert oracle.first_uncovered(exact, got, ppm) == -1
    assert oracle.first_dominated(got) == -1
    assert got.shape[0] <= exact.shape[0]
    if r.paths is not None:
        check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("ppm", [0, 5_000, 100_000])
@pytest.mark.parametrize("B", [256, 4096])
def test_grid_queries(mos, ppm, B):
    for seed in (0, 4):
        g, s, t = gen.config1(seed)
        exact = oracle.solve(g, s, t, 3, flags=FLAGS).costs
        r = mos.mos_solve(mos.Graph.from_gen(g), s, t, batch_width=B, epsilon_ppm=ppm,
                          mem_budget=1 << 30)
        _valid(g, s, t, 3, exact, r, ppm)
        if ppm == 0:
            assert np.array_equal(r.costs.astype(np.int64), exact)


@pytest.mark.parametrize("seed", range(6))
def test_random_multigraphs(mos, seed):
    d = 2 + seed % 3
    g = gen.random_small(9, 28, d, seed=200 + seed, cmax=40)
    G = mos.Graph.from_gen(g)
    for s, t in [(0, 8), (2, 6)]:
        exact = oracle.solve(g, s, t, d, flags=FLAGS).costs
        for ppm in (30_000, 300_000):
            for B in (1, 8):
                _valid(g, s, t, d, exact, mos.mos_solve(G, s, t, batch_width=B, epsilon_ppm=ppm,
                                                        mem_budget=1 << 28), ppm)


def test_stored_fronts_with_less_work(mos):
    # the mid-range ship-grid queries and a 12-objective route, exact fronts stored
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    gm = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gm)
    ship = gen.ship_grid(256, 256, 3, 0)
    G = mos.Graph.from_gen(ship)
    for f in sorted(glob.glob(os.path.join(HERE, "c4mid", "q*.txt.gz")))[:6]:
        h, exact = gm.read_front(f)
        s, t = int(h["start"]), int(h["goal"])
        full = mos.mos_solve(G, s, t, batch_width=1024, costs_only=True)
        apx = mos.mos_solve(G, s, t, batch_width=1024, epsilon_ppm=10_000)
        assert np.array_equal(full.costs.astype(np.int64), exact)
        _valid(ship, s, t, 3, exact, apx, 10_000)
        assert apx.stats["pops"] <= full.stats["pops"]
        print(f"{h['workload']}: front {exact.shape[0]} -> {apx.costs.shape[0]} at 1 %, pops "
              f"{full.stats['pops']} -> {apx.stats['pops']}")
    h, exact = gm.read_front(os.path.join(HERE, "routes", "r4.txt.gz"))
    g, s, t = gen.tmplar_route(4, 12, 0)
    apx = mos.mos_solve(mos.Graph.from_gen(g), s, t, n_objectives=12, batch_width=1024,
                        epsilon_ppm=20_000)
    _valid(g, s, t, 12, exact, apx, 20_000)
    assert apx.costs.shape[0] < exact.shape[0]

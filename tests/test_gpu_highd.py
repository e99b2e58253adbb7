"""GPU path vs the CPU oracle at up to 12 objectives on time-expanded ship
routes shaped like the paper's Table 2 (exact, bit-identical fronts)."""
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


def _check(mos, g, s, t, fronts, ds):
    for r, d in zip(fronts, ds):
        ref = oracle.solve(g, s, t, d)
        assert ref.status == "ok"
        assert np.array_equal(r.costs.astype(np.int64), ref.costs), d
        check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("route,ds,B", [(4, [9, 10, 11, 12], 256), (4, [12], 7),
                                        (1, [8, 9, 10], 512), (3, [5, 6], 1024)])
def test_route_fronts(mos, route, ds, B):
    """One 12-objective graph; each query keeps the first d objectives (Table 1's rule)."""
    g, s, t = gen.tmplar_route(route, 12, 0)
    G = mos.Graph.from_gen(g)
    S = np.full(len(ds), s, dtype=np.int32)
    T = np.full(len(ds), t, dtype=np.int32)
    res = mos.mos_solve_batch(G, S, T, n_objectives=np.array(ds, dtype=np.int32),
                              batch_width=B, mem_budget=4 << 30)
    assert all(st == mos.MOS_OK for st, _ in res)
    _check(mos, g, s, t, [r for _, r in res], ds)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_route_seeds_d12(mos, seed):
    g, s, t = gen.time_expanded_route(8, 2, 12, seed=seed)
    r = mos.mos_solve(mos.Graph.from_gen(g), s, t, batch_width=128, mem_budget=4 << 30)
    _check(mos, g, s, t, [r], [12])


def test_tiny_routes_all_d(mos):
    """Every d from 1 to 12 on a small route, one batched call."""
    g, s, t = gen.time_expanded_route(5, 3, 12, seed=7, windows=6)
    G = mos.Graph.from_gen(g)
    ds = list(range(1, 13))
    res = mos.mos_solve_batch(G, np.full(12, s, np.int32), np.full(12, t, np.int32),
                              n_objectives=np.array(ds, np.int32), batch_width=64,
                              mem_budget=4 << 30)
    assert all(st == mos.MOS_OK for st, _ in res)
    _check(mos, g, s, t, [r for _, r in res], ds)

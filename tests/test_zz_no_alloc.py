"""mos_solve_noalloc (no device allocation; state in the library's static
device array) against mos_solve on the same queries, through the C ABI."""
import ctypes

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def _raw_noalloc(mos, G, s, t, d, cap, **opts):
    """Call the C symbol directly: (status, costs or None, stats dict)."""
    o = mos.make_options(n_objectives=d, **opts)
    buf = np.full((max(cap, 1), d), -7, dtype=np.int32)
    n = ctypes.c_int64(-1)
    st = mos.mos_stats()
    rc = mos.raw.mos_solve_noalloc(G.handle, int(s), int(t), ctypes.byref(o),
                                   buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(cap),
                                   ctypes.byref(n), ctypes.byref(st))
    if rc != mos.MOS_OK:
        return rc, buf, None
    return rc, buf[:n.value].copy(), {f: getattr(st, f) for f, _ in mos.mos_stats._fields_}


def test_two_calls_in_a_row_match_mos_solve(mos):
    # first a 32x32 grid query (front of thousands), then a smaller 12x12 one:
    # the second call must not see anything the first left in the array
    g1, s1, t1 = gen.config1(3)
    g2 = gen.grid_uniform(12, 12, 3, 1, 10, seed=5)
    for g, s, t in ((g1, s1, t1), (g2, 0, g2.n - 1)):
        G = mos.Graph.from_gen(g)
        ref = mos.mos_solve(G, s, t, costs_only=True, mem_budget=1 << 30)
        rc, got, st = _raw_noalloc(mos, G, s, t, 3, cap=ref.costs.shape[0] + 5, batch_width=256)
        assert rc == mos.MOS_OK, mos.raw.mos_last_error()
        assert np.array_equal(got, ref.costs)
        assert st["front"] == ref.costs.shape[0]
        o = oracle.solve(g, s, t, 3)
        assert np.array_equal(got.astype(np.int64), o.costs)


def test_repeated_and_different_objective_counts(mos):
    g, s, t = gen.config1(0)
    G = mos.Graph.from_gen(g)
    for d in (3, 1, 2, 3):
        ref = mos.mos_solve(G, s, t, n_objectives=d, costs_only=True, mem_budget=1 << 30)
        got = mos.mos_solve_noalloc(G, s, t, cap=1 << 15, n_objectives=d, batch_width=1024)
        assert np.array_equal(got.costs, ref.costs), d


def test_front_larger_than_cap_is_rejected(mos):
    g, s, t = gen.config1(0)
    G = mos.Graph.from_gen(g)
    ref = mos.mos_solve(G, s, t, costs_only=True, mem_budget=1 << 30)
    cap = ref.costs.shape[0] - 1
    rc, buf, _ = _raw_noalloc(mos, G, s, t, 3, cap=cap)
    assert rc == mos.MOS_E_INVALID_ARG
    assert np.all(buf == -7)  # nothing written
    assert b"cap" in mos.raw.mos_last_error()


def test_graph_too_large_is_rejected(mos):
    # a 2.5M-node path: its per-node state alone exceeds the array
    n = 2_500_000
    g = gen.from_arcs(n, np.arange(n - 1), np.arange(1, n), np.ones((n - 1, 1), np.int64))
    G = mos.Graph.from_gen(g)
    rc, _, _ = _raw_noalloc(mos, G, 0, n - 1, 1, cap=4)
    assert rc == mos.MOS_E_INVALID_ARG
    assert b"too large" in mos.raw.mos_last_error()


def test_search_outgrowing_the_array_fails_cleanly(mos):
    # the full-size ship grid, corner to corner: far more labels than fit
    g, s, t = gen.config2(0)
    G = mos.Graph.from_gen(g)
    rc, _, _ = _raw_noalloc(mos, G, s, t, 3, cap=1 << 16, batch_width=4096)
    assert rc == mos.MOS_E_LABEL_LIMIT
    # and the array is usable again right after
    g2, s2, t2 = gen.config1(1)
    G2 = mos.Graph.from_gen(g2)
    ref = mos.mos_solve(G2, s2, t2, costs_only=True, mem_budget=1 << 30)
    got = mos.mos_solve_noalloc(G2, s2, t2, cap=1 << 15)
    assert np.array_equal(got.costs, ref.costs)

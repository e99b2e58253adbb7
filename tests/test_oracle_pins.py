"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The oracle (sequential NAMOA*, paper Algorithm 1) is checked against:
  * brute force: every simple start->goal path enumerated by DFS, then the
    minimal distinct cost set (the definition of the problem, paper Section 3);
  * d = 1: the single shortest-path distance (scipy's Dijkstra);
  * the ideal point: per objective, the front's minimum equals the
    single-objective shortest distance;
  * lexicographic extreme points: for every objective order, the
    lexicographically smallest front vector equals a lexicographic Dijkstra
    written here with tuple keys;
  * supported points: for positive weights w, min over the front of w.y equals
    Dijkstra on the scalarised costs w.c;
  * closed forms (diamond chains, identical objectives);
  * metamorphic relations (zero heuristic, node relabelling, objective
    permutation, reversal, scaling, a redundant objective) and the readings of
    the paper's ambiguous points (strict vs weak P tests, eager vs lazy PruneOPEN).
  * the work: the number of extractions equals the count of cost vectors that
    are Pareto-optimal at their node and not heuristic-dominated by the front,
    taken by brute force (NAMOA* with a consistent heuristic extracts exactly
    those).
A mistake such as a dropped prune, a transposed comparison, a wrong heuristic
direction or a wrong cost index breaks at least one of these; the mutant
tests plant such mistakes and check that.
"""
import heapq
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import gen
import oracle
from helpers import check_paths, is_antichain, sort_lex

MODES = [0, oracle.WEAK_P, oracle.LAZY_PRUNEOPEN, oracle.WEAK_P | oracle.LAZY_PRUNEOPEN,
         oracle.ZERO_H]


# ------------------------------------------------------------ independent refs
def brute_front(g, s, t, d):
    """Minimal distinct costs over all simple s->t paths (DFS)."""
    rp, col, cost = g.row_ptr, g.col, g.cost[:, :d].astype(np.int64)
    costs = set()
    if s == t:
        return np.zeros((1, d), dtype=np.int64)
    onpath = np.zeros(g.n, dtype=bool)

    def dfs(u, acc):
        if u == t:
            costs.add(tuple(acc))
            return
        onpath[u] = True
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            if not onpath[v]:
                dfs(v, acc + cost[e])
        onpath[u] = False

    dfs(s, np.zeros(d, dtype=np.int64))
    arr = np.array(sorted(costs), dtype=np.int64).reshape(-1, d)
    keep = []
    for i, y in enumerate(arr):
        dom = np.all(arr <= y, axis=1) & np.any(arr < y, axis=1)
        if not dom.any():
            keep.append(y)
    return sort_lex(np.array(keep, dtype=np.int64).reshape(-1, d))


def scipy_dist(g, w, s):
    """Dijkstra distances from s with arc weights w (float64; exact for small ints)."""
    src = g.arc_sources()
    # parallel arcs: keep the cheapest (csr_matrix would add duplicates)
    order = np.lexsort((w, g.col, src))
    src_o, dst_o, w_o = src[order], g.col[order], w[order]
    first = np.ones(src_o.size, dtype=bool)
    first[1:] = (src_o[1:] != src_o[:-1]) | (dst_o[1:] != dst_o[:-1])
    # zero weights vanish in sparse matrices: shift by a tiny epsilon scaled out later
    eps = 1e-9
    m = sp.csr_matrix((w_o[first].astype(np.float64) + eps, (src_o[first], dst_o[first])),
                      shape=(g.n, g.n))
    dist = dijkstra(m, indices=s)
    return dist


def lex_dijkstra(g, s, t, perm):
    """Lexicographically smallest s->t cost under objective order `perm` (tuple keys)."""
    rp, col = g.row_ptr, g.col
    cost = g.cost[:, list(perm)].astype(np.int64)
    best = {s: tuple([0] * len(perm))}
    pq = [(best[s], s)]
    done = set()
    while pq:
        key, u = heapq.heappop(pq)
        if u in done:
            continue
        done.add(u)
        if u == t:
            return key
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            nk = tuple(a + int(b) for a, b in zip(key, cost[e]))
            if v not in best or nk < best[v]:
                best[v] = nk
                heapq.heappush(pq, (nk, v))
    return None


# ------------------------------------------------------------------- tests
@pytest.mark.parametrize("seed", range(16))
def test_brute_force_random(seed):
    d = 1 + seed % 4
    g = gen.random_small(8, 20, d, seed=seed)
    for s, t in [(0, 7), (2, 5), (4, 4), (6, 1)]:
        ref = brute_front(g, s, t, d)
        for mode in MODES:
            r = oracle.solve(g, s, t, d, flags=mode)
            assert r.status == "ok"
            assert np.array_equal(r.costs, ref), (seed, s, t, mode)
            check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("rows,cols,d", [(2, 2, 2), (3, 3, 3), (3, 4, 2), (4, 4, 3), (4, 5, 2)])
def test_brute_force_grids(rows, cols, d):
    g = gen.grid_uniform(rows, cols, d, 0, 5, seed=rows * 10 + cols)
    ref = brute_front(g, 0, g.n - 1, d)
    for mode in MODES:
        r = oracle.solve(g, 0, g.n - 1, d, flags=mode)
        assert np.array_equal(r.costs, ref), mode


def test_single_objective_is_dijkstra():
    for seed in range(4):
        g, s, t = gen.config1(seed)
        g1 = gen.with_costs(g, g.cost[:, :1])
        r = oracle.solve(g1, s, t, 1)
        dist = scipy_dist(g1, g1.cost[:, 0].astype(np.int64), s)
        assert r.costs.shape == (1, 1)
        assert r.costs[0, 0] == int(round(dist[t]))


@pytest.mark.parametrize("seed", [0, 1])
def test_extreme_and_supported_points_config1(seed):
    g, s, t = gen.config1(seed)
    r = oracle.solve(g, s, t, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN)
    f = r.costs
    assert is_antichain(f)
    assert np.array_equal(f, sort_lex(f))
    # ideal point
    for k in range(3):
        dist = scipy_dist(g, g.cost[:, k].astype(np.int64), s)
        assert f[:, k].min() == int(round(dist[t]))
    # lexicographic extreme for every objective order
    for perm in itertools.permutations(range(3)):
        key = lex_dijkstra(g, s, t, perm)
        fp = f[:, list(perm)]
        assert tuple(int(x) for x in sort_lex(fp)[0]) == key, perm
    # supported points
    rng = np.random.default_rng(seed)
    for _ in range(5):
        w = rng.integers(1, 20, 3)
        dist = scipy_dist(g, (g.cost.astype(np.int64) * w).sum(1), s)
        assert (f * w).sum(1).min() == int(round(dist[t]))
    check_paths(g, s, t, f, r.paths, 3)


def test_extreme_points_ship_grid():
    g, s, t = gen.config2(0, size=64)
    r = oracle.solve(g, s, t)
    f = r.costs
    for perm in itertools.permutations(range(3)):
        key = lex_dijkstra(g, s, t, perm)
        assert tuple(int(x) for x in sort_lex(f[:, list(perm)])[0]) == key
    check_paths(g, s, t, f, r.paths, 3)


@pytest.mark.parametrize("k", [1, 3, 6, 9])
def test_diamond_chain_closed_form(k):
    g, s, t = gen.diamond_chain(k)
    W = 2 ** k - 1
    r = oracle.solve(g, s, t)
    expect = np.array([[x, W - x] for x in range(2 ** k)], dtype=np.int64)
    assert np.array_equal(r.costs, expect)
    check_paths(g, s, t, r.costs, r.paths, 2)


def test_diamond_chain_unit_weights():
    g, s, t = gen.diamond_chain(7, weights=[1] * 7)
    r = oracle.solve(g, s, t)
    expect = np.array([[x, 7 - x] for x in range(8)], dtype=np.int64)
    assert np.array_equal(r.costs, expect)


def test_identical_objectives_singleton():
    g, s, t = gen.config1(2)
    g3 = gen.with_costs(g, np.repeat(g.cost[:, :1], 3, axis=1))
    r = oracle.solve(g3, s, t)
    dist = scipy_dist(g, g.cost[:, 0].astype(np.int64), s)
    assert r.costs.shape == (1, 3) and np.all(r.costs == int(round(dist[t])))


def test_metamorphic_relations():
    g = gen.grid_uniform(9, 9, 3, 1, 10, seed=11)
    s, t = 0, g.n - 1
    base = oracle.solve(g, s, t).costs
    # every reading/mode gives the same cost set
    for mode in MODES:
        assert np.array_equal(oracle.solve(g, s, t, flags=mode).costs, base)
    # node relabelling
    perm = np.random.default_rng(0).permutation(g.n)
    gp = gen.permute_nodes(g, perm)
    assert np.array_equal(oracle.solve(gp, perm[s], perm[t]).costs, base)
    # objective permutation permutes columns
    for p in itertools.permutations(range(3)):
        r = oracle.solve(gen.with_costs(g, g.cost[:, list(p)]), s, t).costs
        assert np.array_equal(r, sort_lex(base[:, list(p)]))
    # reversal on a symmetric graph with swapped endpoints
    assert np.array_equal(oracle.solve(g.reversed(), t, s).costs, base)
    assert np.array_equal(oracle.solve(g, t, s).costs, base)
    # scaling by an integer
    assert np.array_equal(oracle.solve(gen.with_costs(g, g.cost * 3), s, t).costs, base * 3)
    # redundant objective c1 + c2 appended
    c4 = np.concatenate([g.cost, (g.cost[:, 0] + g.cost[:, 1])[:, None]], axis=1)
    r4 = oracle.solve(gen.with_costs(g, c4), s, t).costs
    assert np.array_equal(r4, np.concatenate([base, (base[:, 0] + base[:, 1])[:, None]], 1))
    # the first-n objectives rule: d=2 solves the graph restricted to columns 0, 1
    r2 = oracle.solve(g, s, t, 2).costs
    assert np.array_equal(r2, oracle.solve(gen.with_costs(g, g.cost[:, :2]), s, t).costs)
    assert is_antichain(r2)


def test_edge_cases():
    g = gen.random_small(6, 10, 2, seed=3)
    # start == goal: the single zero vector, empty path
    r = oracle.solve(g, 2, 2)
    assert r.costs.tolist() == [[0, 0]] and len(r.paths[0]) == 0
    # unreachable goal: empty front
    g2 = gen.from_arcs(4, [0, 1], [1, 0], np.ones((2, 2), dtype=np.int64))
    assert oracle.solve(g2, 0, 3).costs.shape == (0, 2)
    # zero-cost cycle and self-loops do not loop forever, parallel arcs pick the best
    g3 = gen.from_arcs(3, [0, 1, 1, 0, 1, 1], [1, 0, 1, 1, 2, 2],
                       np.array([[0, 0], [0, 0], [0, 0], [2, 1], [1, 3], [3, 1]]))
    r3 = oracle.solve(g3, 0, 2)
    assert r3.costs.tolist() == [[1, 3], [3, 1]]
    check_paths(g3, 0, 2, r3.costs, r3.paths, 2)
    # negative costs are rejected
    g4 = gen.from_arcs(2, [0], [1], np.array([[1, 1]]))
    g4.cost[0, 0] = -1
    assert oracle.solve(g4, 0, 1).status == "bad input"


def test_heuristic_is_reverse_dijkstra():
    g, s, t = gen.config1(0)
    h = oracle.heuristic(g, t)
    for k in range(3):
        dist = scipy_dist(g.reversed(), g.reversed().cost[:, k].astype(np.int64), t)
        assert np.array_equal(h[k], np.rint(dist).astype(np.int64))
    # directed: unreachable nodes get the INT64 max marker
    g2 = gen.from_arcs(3, [0, 1], [1, 2], np.ones((2, 1), dtype=np.int64))
    h2 = oracle.heuristic(g2, 0)
    assert h2[0, 0] == 0 and h2[0, 1] == oracle.INF and h2[0, 2] == oracle.INF


@pytest.mark.parametrize("shape,d,seed", [((3, 2, 3), 12, 1), ((2, 3, 3), 11, 2), ((4, 2, 2), 10, 3),
                                          ((3, 3, 2), 9, 4), ((5, 2, 2), 12, 5), ((3, 2, 3), 7, 6)])
def test_brute_force_time_expanded(shape, d, seed):
    """Up to 12 objectives on tiny time-expanded routes (directed, zero-cost
    sink arcs, sideways cycles inside a window)."""
    length, width, windows = shape
    g, s, t = gen.time_expanded_route(length, width, d, seed=seed, windows=windows)
    ref = brute_front(g, s, t, d)
    for mode in MODES:
        r = oracle.solve(g, s, t, d, flags=mode)
        assert r.status == "ok"
        assert np.array_equal(r.costs, ref), mode
        check_paths(g, s, t, r.costs, r.paths, d)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_random_high_d(seed):
    d = 9 + seed % 4
    g = gen.random_small(7, 18, d, seed=100 + seed, cmax=9)
    for s, t in [(0, 6), (3, 1)]:
        ref = brute_front(g, s, t, d)
        r = oracle.solve(g, s, t, d)
        assert np.array_equal(r.costs, ref), (seed, s, t)


def nondominated_costs_per_node(g, s, t, d):
    """For every node v, the distinct minimal costs over all simple s->v paths
    that do not pass through the goal t before their end (DFS; a label at the
    goal is never expanded, so nothing beyond the goal is searched)."""
    rp, col, cost = g.row_ptr, g.col, g.cost[:, :d].astype(np.int64)
    seen = [set() for _ in range(g.n)]
    onpath = np.zeros(g.n, dtype=bool)

    def dfs(u, acc):
        seen[u].add(tuple(int(x) for x in acc))
        if u == t:
            return
        onpath[u] = True
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            if not onpath[v]:
                dfs(v, acc + cost[e])
        onpath[u] = False

    dfs(s, np.zeros(d, dtype=np.int64))
    out = []
    for S in seen:
        a = np.array(sorted(S), dtype=np.int64).reshape(-1, d)
        keep = [y for y in a if not (np.all(a <= y, axis=1) & np.any(a < y, axis=1)).any()]
        out.append(np.array(keep, dtype=np.int64).reshape(-1, d))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_pops_are_the_pareto_optimal_labels(seed):
    """Work pin.  With OPEN in lexicographic order and a consistent heuristic
    (the exact per-objective distance is one, and so is h = 0), every label
    the sequential search extracts is Pareto-optimal at its node and its F is
    not dominated by the final front, and every such cost vector is extracted
    once (paper, Sections 1 and 4: the sequential lexicographic extraction is
    the work-efficiency baseline because each label it extracts is globally
    Pareto-optimal).  So the number of extractions equals a count taken by
    brute force over the simple paths that stop at the goal.  A dropped or
    misplaced prune changes the work but not the front; this pin sees it."""
    d = 1 + seed % 4
    if seed < 10:
        g = gen.random_small(8, 20, d, seed=200 + seed)
        pairs = [(0, 7), (4, 2)]
    else:  # zero-cost sink arcs and cycles inside each time window
        g, s0, t0 = gen.time_expanded_route(3, 2, d, seed=seed, windows=3)
        pairs = [(s0, t0)]
    for s, t in pairs:
        nd = nondominated_costs_per_node(g, s, t, d)
        front = brute_front(g, s, t, d)
        for mode in (0, oracle.LAZY_PRUNEOPEN, oracle.ZERO_H,
                     oracle.ZERO_H | oracle.LAZY_PRUNEOPEN):
            h = (np.zeros((d, g.n), dtype=np.int64) if mode & oracle.ZERO_H
                 else oracle.heuristic(g, t, d))
            want = 0
            for v in range(g.n):
                if nd[v].shape[0] == 0 or (h[:, v] == oracle.INF).any():
                    continue
                F = nd[v] + h[:, v]
                for f in F:
                    dom = (np.all(front <= f, axis=1) & np.any(front < f, axis=1)).any()
                    want += not dom
            r = oracle.solve(g, s, t, d, flags=mode)
            assert np.array_equal(r.costs, front)
            assert r.stats["pops"] == want, (seed, s, t, mode)
            assert r.stats["goal_pops"] == front.shape[0]


@pytest.mark.parametrize("m", [1, 2, 5, 17])
def test_pair_counters_closed_form_on_a_fan(m):
    """The work counters the benches compare against, in closed form.  A fan:
    arcs s -> a_i of cost (i, m-1-i) and a_i -> t of cost (0, 0), i < m.  The
    m goal costs are mutually non-dominated and reach the goal in
    lexicographic order, one per two pops, so every count follows by hand from
    Algorithm 1's procedures (Section 4): the i-th goal candidate meets i
    labels at t (NotDominated over alpha(t)) and i goal labels in P at
    insertion; the i-th goal pop runs Prune(P) and NotDominated(P) over i
    labels each; eager PruneOPEN scans the m-1-i a-labels still open, and the
    lazy form instead checks each popped label against P (i labels for a_i and
    for t_i).  Nothing dominates, so no loop breaks early."""
    n = m + 2
    s, t = 0, m + 1
    src = [s] * m + list(range(1, m + 1))
    dst = list(range(1, m + 1)) + [t] * m
    cost = [[i, m - 1 - i] for i in range(m)] + [[0, 0]] * m
    g = gen.graphs.from_arcs(n, np.array(src), np.array(dst), np.array(cost))
    tri = m * (m - 1) // 2
    want = {0: dict(frontier_pairs=tri, p_pairs=3 * tri, open_pairs=tri),
            oracle.LAZY_PRUNEOPEN: dict(frontier_pairs=tri, p_pairs=5 * tri, open_pairs=0)}
    for mode, counts in want.items():
        r = oracle.solve(g, s, t, 2, flags=mode)
        assert np.array_equal(r.costs, np.array(cost[:m], dtype=np.int64))
        got = {k: r.stats[k] for k in counts}
        assert got == counts, (m, mode)
        assert r.stats["pops"] == 2 * m + 1
        assert r.stats["goal_pops"] == m
        assert r.stats["candidates"] == 2 * m
        assert r.stats["killed"] == 0 and r.stats["pruned"] == 0
        assert r.stats["max_alpha"] == m - 1

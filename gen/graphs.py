"""Seeded synthetic instances for the multi-objective shortest-path search.

This module only *builds inputs*: graphs in CSR form with non-negative int32
cost vectors per arc, and start/goal queries.  It contains none of the search
arithmetic, so both the CPU oracle (test infrastructure) and the GPU library
consume exactly the same bytes from it.

Problem statement being instantiated (paper, Section 3): a graph G=(V,E,c)
where every edge carries a non-negative cost vector of length d.  The paper's
own workloads (TMPLAR ship-routing graphs, Tables 1-2; ERA5 weather) are not
available, so the graphs below are stand-ins: smooth-field grids shaped like
ship routing, and random geometric graphs shaped like road networks.

Every generator uses ``numpy.random.default_rng(seed)`` and a fixed draw order
(documented per function), so the same seed always gives the same bytes.
Rounding uses ``np.rint`` in float64 (round half to even).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

INT32_MAX = 2**31 - 1


@dataclasses.dataclass
class Graph:
    """Directed graph in CSR form.

    row_ptr: int64[n+1]; col: int32[E] (arc targets); cost: int32[E, D]
    (arc-major: cost[e, k] is objective k of arc e).  Arcs of node u are
    row_ptr[u]..row_ptr[u+1]-1, sorted by target id.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    cost: np.ndarray
    name: str = ""
    coords: np.ndarray | None = None  # optional node positions (float64[n,2])

    @property
    def n_arcs(self) -> int:
        return int(self.col.shape[0])

    @property
    def D(self) -> int:
        return int(self.cost.shape[1])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col, self.cost):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]

    def arc_sources(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr))

    def reversed(self) -> "Graph":
        """The transpose graph (every arc u->v becomes v->u, same cost)."""
        src = self.arc_sources()
        return from_arcs(self.n, self.col, src, self.cost, name=self.name + "^T")


def from_arcs(n: int, src, dst, cost, name: str = "", coords=None) -> Graph:
    """CSR from a directed arc list; arcs are ordered by (source, target, input order)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    cost = np.asarray(cost)
    if cost.ndim == 1:
        cost = cost[:, None]
    if cost.min(initial=0) < 0 or cost.max(initial=0) > INT32_MAX:
        raise ValueError("costs must lie in [0, INT32_MAX]")
    order = np.lexsort((np.arange(src.size), dst, src))
    src, dst, cost = src[order], dst[order], cost[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32),
                 cost=np.ascontiguousarray(cost.astype(np.int32)), name=name,
                 coords=coords)


def from_edges(n: int, u, v, cost, name: str = "", coords=None) -> Graph:
    """CSR from an undirected edge list: each edge becomes two arcs sharing one cost vector."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    cost = np.asarray(cost)
    if cost.ndim == 1:
        cost = cost[:, None]
    return from_arcs(n, np.concatenate([u, v]), np.concatenate([v, u]),
                     np.concatenate([cost, cost]), name=name, coords=coords)


# --------------------------------------------------------------------------
# Plain single query: 32x32 4-connected grid, d=3, costs U{1..10}
# --------------------------------------------------------------------------

def grid4_edges(rows: int, cols: int):
    """Canonical edge order: horizontal edges row-major, then vertical edges row-major."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols - 1), indexing="ij")
    hu = (r * cols + c).ravel()
    hv = hu + 1
    r, c = np.meshgrid(np.arange(rows - 1), np.arange(cols), indexing="ij")
    vu = (r * cols + c).ravel()
    vv = vu + cols
    return np.concatenate([hu, vu]), np.concatenate([hv, vv])


def grid_uniform(rows: int = 32, cols: int = 32, d: int = 3, lo: int = 1, hi: int = 10,
                 seed: int = 0) -> Graph:
    """4-connected grid, node id = cols*row + col, one cost vector per undirected
    edge drawn as ``rng.integers(lo, hi+1, (n_edges, d))`` in canonical edge order."""
    rng = np.random.default_rng(seed)
    u, v = grid4_edges(rows, cols)
    cost = rng.integers(lo, hi + 1, size=(u.size, d))
    rr, cc = np.divmod(np.arange(rows * cols), cols)
    return from_edges(rows * cols, u, v, cost, name=f"grid{rows}x{cols}_d{d}_s{seed}",
                      coords=np.stack([cc, rr], 1).astype(np.float64))


def config1(seed: int = 0):
    """32x32 4-connected grid, d=3, costs U{1..10}; start (0,0), goal (31,31)."""
    g = grid_uniform(32, 32, 3, 1, 10, seed)
    return g, 0, 32 * 32 - 1


# --------------------------------------------------------------------------
# Ship-routing-shaped grid: 256x256, 8-connected, smooth-field costs
# --------------------------------------------------------------------------

def grid8_edges(rows: int, cols: int):
    """Edges of an 8-connected grid with their lengths (1 or sqrt 2).

    Order: horizontal, vertical, diagonal down-right, diagonal down-left; each row-major."""
    us, vs, ls = [], [], []
    r, c = np.meshgrid(np.arange(rows), np.arange(cols - 1), indexing="ij")
    a = (r * cols + c).ravel(); us.append(a); vs.append(a + 1); ls.append(np.ones(a.size))
    r, c = np.meshgrid(np.arange(rows - 1), np.arange(cols), indexing="ij")
    a = (r * cols + c).ravel(); us.append(a); vs.append(a + cols); ls.append(np.ones(a.size))
    r, c = np.meshgrid(np.arange(rows - 1), np.arange(cols - 1), indexing="ij")
    a = (r * cols + c).ravel(); us.append(a); vs.append(a + cols + 1)
    ls.append(np.full(a.size, np.sqrt(2.0)))
    r, c = np.meshgrid(np.arange(rows - 1), np.arange(1, cols), indexing="ij")
    a = (r * cols + c).ravel(); us.append(a); vs.append(a + cols - 1)
    ls.append(np.full(a.size, np.sqrt(2.0)))
    return np.concatenate(us), np.concatenate(vs), np.concatenate(ls)


def smooth_fields(rows: int, cols: int, d: int, rng, n_bumps: int = 16):
    """d fields, each a sum of Gaussian bumps min-max normalised to [0, 2].

    Draw order per field k: centres U[0,size)^2 as (n_bumps, 2) [x, y],
    widths U[8, 48] (n_bumps), amplitudes U[0.5, 1.5] (n_bumps).
    Field value is evaluated at node centres (x = column, y = row)."""
    yy, xx = np.meshgrid(np.arange(rows, dtype=np.float64),
                         np.arange(cols, dtype=np.float64), indexing="ij")
    fields = np.empty((d, rows * cols))
    for k in range(d):
        mu = rng.uniform(0.0, float(max(rows, cols)), size=(n_bumps, 2))
        sig = rng.uniform(8.0, 48.0, size=n_bumps)
        amp = rng.uniform(0.5, 1.5, size=n_bumps)
        f = np.zeros((rows, cols))
        for b in range(n_bumps):
            f += amp[b] * np.exp(-((xx - mu[b, 0]) ** 2 + (yy - mu[b, 1]) ** 2)
                                 / (2.0 * sig[b] ** 2))
        f = f.ravel()
        lo, hi = f.min(), f.max()
        fields[k] = 2.0 * (f - lo) / (hi - lo) if hi > lo else 0.0
    return fields


def ship_grid(rows: int = 256, cols: int = 256, d: int = 3, seed: int = 0) -> Graph:
    """8-connected grid; c_k(u,v) = rint(100 * len * (1 + (F_k(u) + F_k(v)) / 2))."""
    rng = np.random.default_rng(seed)
    fields = smooth_fields(rows, cols, d, rng)
    u, v, length = grid8_edges(rows, cols)
    cost = np.rint(100.0 * length[:, None] * (1.0 + (fields[:, u].T + fields[:, v].T) / 2.0))
    rr, cc = np.divmod(np.arange(rows * cols), cols)
    return from_edges(rows * cols, u, v, cost.astype(np.int64),
                      name=f"ship{rows}x{cols}_d{d}_s{seed}",
                      coords=np.stack([cc, rr], 1).astype(np.float64))


def config2(seed: int = 0, size: int = 256):
    """256x256 ship-shaped grid, d=3; start (0,0), goal (size-1,size-1)."""
    g = ship_grid(size, size, 3, seed)
    return g, 0, size * size - 1


def ship_queries(rows: int, cols: int, nq: int, seed: int, dmin: int = 10, dmax: int = 400):
    """Start/goal pairs whose Manhattan distance D ~ U{dmin..dmax}.

    Per query: draw D, then s uniformly; t uniformly among nodes at Manhattan
    distance exactly D from s (s is redrawn while there is none)."""
    rng = np.random.default_rng(seed)
    rr, cc = np.divmod(np.arange(rows * cols), cols)
    starts, goals = np.empty(nq, np.int32), np.empty(nq, np.int32)
    for i in range(nq):
        D = int(rng.integers(dmin, dmax + 1))
        while True:
            s = int(rng.integers(0, rows * cols))
            sr, sc = divmod(s, cols)
            cand = np.flatnonzero(np.abs(rr - sr) + np.abs(cc - sc) == D)
            if cand.size:
                break
        starts[i] = s
        goals[i] = int(cand[rng.integers(0, cand.size)])
    return starts, goals


def config4(seed: int = 0, nq: int = 512, size: int = 256):
    """Batch of nq queries on the seed-0 ship grid (the graph uses seed 0; the
    query draw uses ``seed + 1000``)."""
    g = ship_grid(size, size, 3, 0)
    s, t = ship_queries(size, size, nq, seed + 1000, 10, min(400, 2 * (size - 1)))
    return g, s, t


# --------------------------------------------------------------------------
# Road-like random geometric graphs (symmetric k-NN)
# --------------------------------------------------------------------------

def knn_edges(points: np.ndarray, k: int):
    """Undirected edges {u,v} where v is among u's k nearest neighbours or vice versa.

    Returned with u < v, sorted lexicographically."""
    from scipy.spatial import cKDTree

    tree = cKDTree(points)
    _, idx = tree.query(points, k=k + 1)
    n = points.shape[0]
    u = np.repeat(np.arange(n, dtype=np.int64), k)
    v = idx[:, 1:].ravel().astype(np.int64)
    a, b = np.minimum(u, v), np.maximum(u, v)
    key = np.unique(a * n + b)
    return key // n, key % n


def components(n: int, u, v) -> np.ndarray:
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    m = coo_matrix((np.ones(u.size), (u, v)), shape=(n, n))
    return connected_components(m, directed=False)[1]


def geometric_graph(n: int, k: int, d: int, seed: int):
    """n points U[0,1)^2 (drawn first, as ``rng.random((n, 2))``), symmetric k-NN.

    c1 = rint(1e4 * euclidean length); for k = 2..d, c_k = rint(c1 * u_k) with
    u_k ~ U[0.5, 2] per edge (drawn as one ``(n_edges, d-1)`` array after the points).
    Returns (graph, rng, component labels)."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    u, v = knn_edges(pts, k)
    length = np.linalg.norm(pts[u] - pts[v], axis=1)
    c1 = np.rint(1e4 * length)
    mult = rng.uniform(0.5, 2.0, size=(u.size, d - 1))
    cost = np.concatenate([c1[:, None], np.rint(c1[:, None] * mult)], axis=1)
    g = from_edges(n, u, v, cost.astype(np.int64), name=f"rgg{n}_k{k}_d{d}_s{seed}", coords=pts)
    return g, rng, components(n, u, v)


def far_pair(g: Graph, comp: np.ndarray, rng, min_dist: float):
    """s, t drawn uniformly until |s - t| >= min_dist and both lie in the giant component."""
    giant = np.bincount(comp).argmax()
    while True:
        s, t = (int(x) for x in rng.integers(0, g.n, size=2))
        if comp[s] != giant or comp[t] != giant:
            continue
        if np.linalg.norm(g.coords[s] - g.coords[t]) >= min_dist:
            return s, t


def config3(seed: int = 0, n: int = 200_000):
    """Road-like single query: 6-NN geometric graph, d=4, |s-t| >= 0.7."""
    g, rng, comp = geometric_graph(n, 6, 4, seed)
    s, t = far_pair(g, comp, rng, 0.7)
    return g, s, t


def config5_graph(seed: int = 0, n: int = 1_000_000):
    """Served workload graph: 8-NN geometric graph with 5 stored objectives."""
    g, rng, comp = geometric_graph(n, 8, 5, seed)
    return g, rng, comp


def served_queries(g: Graph, comp: np.ndarray, nq: int, seed: int, dmin: int = 3, dmax: int = 5):
    """nq random distinct (s, t) pairs in the giant component, each with a number
    of objectives d ~ U{dmin..dmax} (the first d stored objectives are used)."""
    rng = np.random.default_rng(seed + 5000)
    giant = np.bincount(comp).argmax()
    nodes = np.flatnonzero(comp == giant)
    s = nodes[rng.integers(0, nodes.size, nq)]
    t = nodes[rng.integers(0, nodes.size, nq)]
    same = s == t
    while same.any():
        t[same] = nodes[rng.integers(0, nodes.size, int(same.sum()))]
        same = s == t
    dq = rng.integers(dmin, dmax + 1, nq)
    return s.astype(np.int32), t.astype(np.int32), dq.astype(np.int32)


def c5_parity_queries(g: Graph, comp: np.ndarray, nq: int, seed: int):
    """nq uniformly random distinct (s, t) pairs in the giant component with
    the objective count stratified: queries i = 0, 3, 6, ... use d = 3, then
    d = 4 and d = 5 in turn (the first d stored objectives)."""
    rng = np.random.default_rng(seed + 8000)
    giant = np.bincount(comp).argmax()
    nodes = np.flatnonzero(comp == giant)
    s = nodes[rng.integers(0, nodes.size, nq)]
    t = nodes[rng.integers(0, nodes.size, nq)]
    same = s == t
    while same.any():
        t[same] = nodes[rng.integers(0, nodes.size, int(same.sum()))]
        same = s == t
    dq = 3 + np.arange(nq) % 3
    return s.astype(np.int32), t.astype(np.int32), dq.astype(np.int32)


def local_queries(g: Graph, comp: np.ndarray, nq: int, seed: int, radius: float,
                  dmin: int = 3, dmax: int = 5):
    """nq (s, t, d) queries in the giant component with t drawn uniformly among
    the nodes within Euclidean distance `radius` of s (t != s), d ~ U{dmin..dmax}.
    The tractable stand-in for random pairs on large geometric graphs."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed + 6000)
    giant = np.bincount(comp).argmax()
    nodes = np.flatnonzero(comp == giant)
    tree = cKDTree(g.coords)
    S, T = np.empty(nq, np.int32), np.empty(nq, np.int32)
    i = 0
    while i < nq:
        s = int(nodes[rng.integers(0, nodes.size)])
        near = [x for x in tree.query_ball_point(g.coords[s], radius) if x != s and comp[x] == giant]
        if not near:
            continue
        S[i], T[i] = s, int(near[rng.integers(0, len(near))])
        i += 1
    dq = rng.integers(dmin, dmax + 1, nq).astype(np.int32)
    return S, T, dq


def poisson_arrivals(nq: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed + 7000)
    return np.cumsum(rng.exponential(1.0 / rate, nq))


# --------------------------------------------------------------------------
# Tiny graphs and gadgets (for brute-force and closed-form checks)
# --------------------------------------------------------------------------

def random_small(n: int, m: int, d: int, seed: int, cmax: int = 6, zero_frac: float = 0.15,
                 self_loops: bool = True):
    """Random directed multigraph: m arcs with uniform endpoints (parallel arcs and,
    optionally, self-loops allowed); costs U{0..cmax} with an extra fraction of
    all-zero cost vectors."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    if not self_loops:
        dst = np.where(dst == src, (dst + 1) % n, dst)
    cost = rng.integers(0, cmax + 1, (m, d))
    zero = rng.random(m) < zero_frac
    cost[zero] = 0
    return from_arcs(n, src, dst, cost, name=f"rand{n}_{m}_d{d}_s{seed}")


def diamond_chain(k: int, weights=None):
    """k diamonds in series.  Diamond i joins node 2i to node 2i+2 through two
    middle branches: an upper one through node 2i+1 costing (w_i, 0) and a lower
    one through an extra node costing (0, w_i) (each branch cost sits on its
    first arc; the second arc costs 0).  Default w_i = 2**i.

    The set of path costs is {(x, W - x)} for x ranging over subset sums of w,
    with W = sum(w); with w_i = 2**i that is every x in 0..2**k - 1."""
    if weights is None:
        weights = [2 ** i for i in range(k)]
    src, dst, cost = [], [], []
    n_main = 2 * k + 1
    extra = n_main
    for i, w in enumerate(weights):
        a, mid, b = 2 * i, 2 * i + 1, 2 * i + 2
        src += [a, mid]; dst += [mid, b]; cost += [(w, 0), (0, 0)]
        src += [a, extra]; dst += [extra, b]; cost += [(0, w), (0, 0)]
        extra += 1
    n = extra
    g = from_arcs(n, src, dst, np.array(cost), name=f"diamonds{k}")
    return g, 0, 2 * k


def permute_nodes(g: Graph, perm: np.ndarray) -> Graph:
    """Relabel node u as perm[u]."""
    src = perm[g.arc_sources()]
    dst = perm[g.col]
    return from_arcs(g.n, src, dst, g.cost, name=g.name + "^perm")


def with_costs(g: Graph, cost: np.ndarray) -> Graph:
    """Same topology, new arc-major cost matrix."""
    return Graph(n=g.n, row_ptr=g.row_ptr.copy(), col=g.col.copy(),
                 cost=np.ascontiguousarray(np.asarray(cost).astype(np.int32)),
                 name=g.name + "^c", coords=g.coords)


def overflow_bound_ok(g: Graph) -> bool:
    """2 * sum_e c_k(e) + max_e c_k(e) < INT32_MAX for every objective k."""
    c = g.cost.astype(np.int64)
    return bool(np.all(2 * c.sum(0) + c.max(0, initial=0) < INT32_MAX))


# --------------------------------------------------------------------------
# Time-expanded ship routes with up to 12 objectives (Tables 1-2 shapes)
# --------------------------------------------------------------------------

# Spatial corridors (cells along the route x cells across) sized so that, with
# 10 time windows per cell and one goal sink, the node counts are close to the
# five routes of Table 2 (201 to 1,610 nodes).
ROUTE_SHAPES = {1: (16, 3), 2: (40, 4), 3: (23, 2), 4: (10, 2), 5: (26, 3)}
# The largest objective count Table 2 reports for each route.
ROUTE_MAX_OBJECTIVES = {1: 12, 2: 4, 3: 12, 4: 12, 5: 6}


def wave_fields(length: int, width: int, windows: int, rng, n_bumps: int = 6):
    """Three time-varying fields over the corridor, each in [0, 1]: wave height,
    wave period and wave direction (as a fraction of a full turn).

    Each field is a sum of Gaussian bumps drifting with constant velocity.
    Draw order per field: centres (n_bumps, 2) as [along, across] with along
    U[0, length) and across U[0, width); velocities (n_bumps, 2) U[-1, 1] cells
    per window; widths U[1, 0.5 * length + 1]; amplitudes U[0.5, 1.5].  The
    field is min-max normalised over all (cell, window) points.
    Returns float64[3, windows, length * width] (cell id = along * width + across)."""
    a, c = np.meshgrid(np.arange(length, dtype=np.float64),
                       np.arange(width, dtype=np.float64), indexing="ij")
    a, c = a.ravel(), c.ravel()
    out = np.empty((3, windows, length * width))
    for f in range(3):
        mu = rng.uniform(0.0, 1.0, size=(n_bumps, 2)) * np.array([length, width])
        vel = rng.uniform(-1.0, 1.0, size=(n_bumps, 2))
        sig = rng.uniform(1.0, 0.5 * length + 1.0, size=n_bumps)
        amp = rng.uniform(0.5, 1.5, size=n_bumps)
        for t in range(windows):
            v = np.zeros(length * width)
            for b in range(n_bumps):
                ca, cc = mu[b] + t * vel[b]
                v += amp[b] * np.exp(-((a - ca) ** 2 + (c - cc) ** 2) / (2.0 * sig[b] ** 2))
            out[f, t] = v
        lo, hi = out[f].min(), out[f].max()
        out[f] = (out[f] - lo) / (hi - lo) if hi > lo else 0.0
    return out


def time_expanded_route(length: int, width: int, d: int = 12, seed: int = 0,
                        windows: int = 10) -> tuple[Graph, int, int]:
    """Directed spatio-temporal ship-routing graph with d <= 12 objectives.

    The spatial part is a corridor of length x width cells from an origin cell
    (along 0, middle column) to a destination cell (along length-1, middle
    column); every cell is expanded into `windows` time windows (Section 6.1
    expands each node into 10).  Node (cell, window) has id cell * windows +
    window; the last id is a goal sink.  From (u, t) there is an arc to (v, t)
    (fast passage) and, if t + 1 < windows, to (v, t + 1) (slow passage), for
    every cell v that is an 8-neighbour of u not behind it along the corridor
    (same or next along index).  Every (destination, t) has a zero-cost arc to
    the sink.  The start is (origin, window 0), the goal the sink.

    Objectives follow the order of Table 1 (the first d are kept): distance,
    fuel, roll, pitch, vertical acceleration, horizontal acceleration,
    vertical bending moment, vertical shear force, wave height, wave period,
    relative wave bearing, random.  With len in {1, sqrt 2}, H, P, W the wave
    height, period and direction fields averaged over the arc's two cells at
    the departure window, r = |cos(2 pi W - bearing)| the relative bearing,
    s = 2 for a fast and 1 for a slow passage:
      distance  rint(100 len)
      fuel      rint(100 len s (1 + H r))
      roll      rint(100 len (0.2 + H (1 - r) + 0.3 P))
      pitch     rint(100 len (0.2 + H r + 0.3 (1 - P)))
      vert acc  rint(100 len (0.1 + s H (0.5 + 0.5 r)))
      horz acc  rint(100 len (0.1 + s H (1 - 0.5 r)))
      VBM       rint(100 len (0.1 + H (1 - P) + 0.2 s))
      VSF       rint(100 len (0.1 + H P + 0.1 s r))
      wave hgt  rint(100 len H)
      wave per  rint(100 len P)
      rel bear  rint(100 len r)
      random    U{0..100} per arc (drawn in arc order)
    Draw order: the three fields (``wave_fields``), then the random objective.
    Returns (graph, start, goal)."""
    if not 1 <= d <= 12:
        raise ValueError("d must lie in [1, 12]")
    rng = np.random.default_rng(seed)
    H, P, W = wave_fields(length, width, windows, rng)
    ncell = length * width
    src_c, dst_c, dlen, bear = [], [], [], []
    for i in range(length):
        for j in range(width):
            for di in (0, 1):
                for dj in (-1, 0, 1):
                    if di == 0 and dj == 0:
                        continue
                    i2, j2 = i + di, j + dj
                    if i2 >= length or not 0 <= j2 < width:
                        continue
                    src_c.append(i * width + j)
                    dst_c.append(i2 * width + j2)
                    dlen.append(np.hypot(di, dj))
                    bear.append(np.arctan2(dj, di))
    src_c, dst_c = np.array(src_c), np.array(dst_c)
    dlen, bear = np.array(dlen), np.array(bear)
    src, dst, cols = [], [], []
    for t in range(windows):
        h = 0.5 * (H[t, src_c] + H[t, dst_c])
        p = 0.5 * (P[t, src_c] + P[t, dst_c])
        r = np.abs(np.cos(2.0 * np.pi * 0.5 * (W[t, src_c] + W[t, dst_c]) - bear))
        for t2, s in ((t, 2.0), (t + 1, 1.0)):
            if t2 >= windows:
                continue
            L = 100.0 * dlen
            c = np.stack([
                L, L * s * (1 + h * r), L * (0.2 + h * (1 - r) + 0.3 * p),
                L * (0.2 + h * r + 0.3 * (1 - p)), L * (0.1 + s * h * (0.5 + 0.5 * r)),
                L * (0.1 + s * h * (1 - 0.5 * r)), L * (0.1 + h * (1 - p) + 0.2 * s),
                L * (0.1 + h * p + 0.1 * s * r), L * h, L * p, L * r,
                np.zeros_like(L)], axis=1)
            src.append(src_c * windows + t)
            dst.append(dst_c * windows + t2)
            cols.append(c)
    sink = ncell * windows
    dest_cell = (length - 1) * width + width // 2
    src.append(dest_cell * windows + np.arange(windows))
    dst.append(np.full(windows, sink))
    cols.append(np.zeros((windows, 12)))
    src, dst = np.concatenate(src), np.concatenate(dst)
    cost = np.rint(np.concatenate(cols))
    cost[: -windows, 11] = rng.integers(0, 101, size=src.size - windows)
    start = (width // 2) * windows
    g = from_arcs(sink + 1, src, dst, cost[:, :d].astype(np.int64),
                  name=f"route{length}x{width}x{windows}_d{d}_s{seed}")
    return g, int(start), int(sink)


def tmplar_route(route: int, d: int = 12, seed: int = 0):
    """A time-expanded route shaped like route `route` (1..5) of Table 2."""
    length, width = ROUTE_SHAPES[route]
    return time_expanded_route(length, width, d, seed)

"""CPU oracle for the exact multi-objective shortest-path search.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the product library.  It
shares no code with the GPU path.

``solve`` runs sequential NAMOA* as laid out in the paper's Algorithm 1 (see
``namoa.cpp``); ``heuristic`` runs the per-objective reverse Dijkstra that
supplies its admissible heuristic (paper, Section 4).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "namoa.cpp")
_SRCS = [_SRC, os.path.join(_HERE, "necessary.cpp")]
_LIB = os.path.join(_HERE, "liboracle.so")

ZERO_H = 1
WEAK_P = 2
LAZY_PRUNEOPEN = 4

STATUS = {0: "ok", 1: "bad input", 2: "label limit", 3: "time limit"}
STAT_NAMES = ["pops", "goal_pops", "candidates", "unreachable", "frontier_pairs", "p_pairs",
              "open_pairs", "inserted", "pruned", "killed", "max_open", "max_alpha"]
INF = np.iinfo(np.int64).max


def build(force: bool = False) -> str:
    """Compile namoa.cpp and necessary.cpp with g++ into liboracle.so (next to this file)."""
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_namoa.restype = ctypes.c_void_p
        lib.oracle_namoa.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p, i32p, i32p,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int64, ctypes.c_double]
        lib.oracle_namoa_ex.restype = ctypes.c_void_p
        lib.oracle_namoa_ex.argtypes = lib.oracle_namoa.argtypes + [ctypes.c_int64]
        lib.oracle_namoa_eps.restype = ctypes.c_void_p
        lib.oracle_namoa_eps.argtypes = lib.oracle_namoa.argtypes + [ctypes.c_int64,
                                                                     ctypes.c_int64]
        lib.oracle_first_uncovered.restype = ctypes.c_int64
        lib.oracle_first_uncovered.argtypes = [ctypes.c_int64, i64p, ctypes.c_int64, i64p,
                                               ctypes.c_int, ctypes.c_int64]
        lib.oracle_open_min.argtypes = [ctypes.c_void_p, i64p]
        lib.oracle_first_dominated.restype = ctypes.c_int64
        lib.oracle_first_dominated.argtypes = [ctypes.c_int64, ctypes.c_int, i64p]
        lib.oracle_lex_dijkstra.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p,
                                            i32p, i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            i32p, i64p]
        lib.oracle_status.argtypes = [ctypes.c_void_p]
        lib.oracle_size.restype = ctypes.c_int64
        lib.oracle_size.argtypes = [ctypes.c_void_p]
        lib.oracle_costs.argtypes = [ctypes.c_void_p, i64p]
        lib.oracle_path_len.restype = ctypes.c_int64
        lib.oracle_path_len.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_path.argtypes = [ctypes.c_void_p, ctypes.c_int64, i32p]
        lib.oracle_stats.argtypes = [ctypes.c_void_p, i64p, ctypes.POINTER(ctypes.c_double)]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_heuristic.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p, i32p,
                                         i32p, ctypes.c_int, ctypes.c_int, i64p]
        lib.oracle_dijkstra.argtypes = [ctypes.c_int, i64p, i32p, i64p, ctypes.c_int, i64p]
        _lib = lib
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


@dataclasses.dataclass
class Front:
    status: str
    costs: np.ndarray          # int64[size, d], lexicographically ascending
    paths: list                # list of int32 arc-id arrays
    stats: dict
    # after an early stop (time or extraction limit): F of the smallest label
    # left in OPEN.  The front so far is then the part of the final front that
    # is lexicographically below it (see prefix_bound).
    open_min: np.ndarray | None = None


def _arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    cost = np.ascontiguousarray(g.cost, dtype=np.int32)
    return rp, col, cost


def solve(g, s: int, t: int, d: int | None = None, flags: int = 0, label_limit: int = 0,
          time_limit: float = 0.0, pop_limit: int = 0, want_paths: bool = True,
          eps_ppm: int = 0) -> Front:
    """Exact Pareto front of s->t costs over the first d objectives of g.

    With a time limit or an extraction limit (pop_limit: labels taken from
    OPEN) the search may stop early (status "time limit"); the result then
    holds the goal front so far and ``open_min``.  eps_ppm > 0 runs the
    approximate mode: tests against the goal front by (1 + eps)-dominance,
    eps = eps_ppm / 10^6 (the result covers the exact front within 1 + eps)."""
    lib = _load()
    d = g.D if d is None else d
    rp, col, cost = _arrays(g)
    r = lib.oracle_namoa_eps(g.n, g.n_arcs, g.D, _ptr(rp, ctypes.c_int64),
                             _ptr(col, ctypes.c_int32), _ptr(cost, ctypes.c_int32), int(s), int(t),
                             int(d), int(flags), int(label_limit), float(time_limit),
                             int(pop_limit), int(eps_ppm))
    try:
        st = STATUS[lib.oracle_status(r)]
        n = lib.oracle_size(r)
        costs = np.zeros((n, d), dtype=np.int64)
        if n:
            lib.oracle_costs(r, _ptr(costs, ctypes.c_int64))
        paths = []
        for i in range(n if want_paths else 0):
            ln = lib.oracle_path_len(r, i)
            p = np.zeros(ln, dtype=np.int32)
            if ln:
                lib.oracle_path(r, i, _ptr(p, ctypes.c_int32))
            paths.append(p)
        sv = np.zeros(len(STAT_NAMES), dtype=np.int64)
        secs = ctypes.c_double()
        lib.oracle_stats(r, _ptr(sv, ctypes.c_int64), ctypes.byref(secs))
        stats = dict(zip(STAT_NAMES, (int(x) for x in sv)))
        stats["search_seconds"] = secs.value
        stats["front"] = int(n)
        om = np.zeros(d, dtype=np.int64)
        open_min = om if lib.oracle_open_min(r, _ptr(om, ctypes.c_int64)) else None
    finally:
        lib.oracle_free(r)
    return Front(st, costs, paths, stats, open_min)


def lex_less(a, b) -> bool:
    """a < b in lexicographic order (objective 0 first)."""
    for x, y in zip(a, b):
        if x != y:
            return x < y
    return False


def prefix_bound(front_so_far: Front):
    """For an early-stopped search: (bound, rows) where bound is the F of the
    smallest label left in OPEN and rows are the goal-front vectors found so
    far that are lexicographically below it.  Any exact front of the same
    query restricted to the vectors below `bound` must equal `rows`."""
    b = front_so_far.open_min
    rows = [r for r in front_so_far.costs if lex_less(r, b)]
    return b, np.array(rows, dtype=np.int64).reshape(-1, front_so_far.costs.shape[1])


def lex_dijkstra(g, s: int, t: int, perm, d: int | None = None):
    """Cost vector (original objective order) of the lexicographically shortest
    s->t path with objectives compared in the order perm; None if t is
    unreachable."""
    lib = _load()
    d = len(perm) if d is None else d
    rp, col, cost = _arrays(g)
    pm = np.ascontiguousarray(perm, dtype=np.int32)
    out = np.zeros(d, dtype=np.int64)
    rc = lib.oracle_lex_dijkstra(g.n, g.n_arcs, g.D, _ptr(rp, ctypes.c_int64),
                                 _ptr(col, ctypes.c_int32), _ptr(cost, ctypes.c_int32), int(s),
                                 int(t), int(d), _ptr(pm, ctypes.c_int32), _ptr(out, ctypes.c_int64))
    if rc < 0:
        raise ValueError("bad lex_dijkstra input")
    return tuple(int(x) for x in out) if rc == 1 else None


def scalar_dijkstra(g, s: int, w) -> np.ndarray:
    """Shortest distances from s under the scalar arc cost sum_k w[k] * c_k(e)."""
    lib = _load()
    rp, col, cost = _arrays(g)
    w = np.asarray(w, dtype=np.int64)
    we = np.ascontiguousarray(cost[:, :len(w)].astype(np.int64) @ w)
    dist = np.zeros(g.n, dtype=np.int64)
    if lib.oracle_dijkstra(g.n, _ptr(rp, ctypes.c_int64), _ptr(col, ctypes.c_int32),
                           _ptr(we, ctypes.c_int64), int(s), _ptr(dist, ctypes.c_int64)):
        raise ValueError("bad dijkstra input")
    return dist


def heuristic(g, goal: int, d: int | None = None) -> np.ndarray:
    """h[k, v] = shortest v->goal distance under objective k (INT64 max if unreachable)."""
    lib = _load()
    d = g.D if d is None else d
    rp, col, cost = _arrays(g)
    h = np.zeros((d, g.n), dtype=np.int64)
    rc = lib.oracle_heuristic(g.n, g.n_arcs, g.D, _ptr(rp, ctypes.c_int64),
                              _ptr(col, ctypes.c_int32), _ptr(cost, ctypes.c_int32), int(goal),
                              int(d), _ptr(h, ctypes.c_int64))
    if rc:
        raise ValueError("bad heuristic input")
    return h


def first_dominated(front) -> int:
    """For rows in lexicographically ascending order: -1 when they are mutually
    non-dominated and distinct, else the index of the first row that an
    earlier row weakly dominates (-2: rows not ascending)."""
    lib = _load()
    f = np.ascontiguousarray(front, dtype=np.int64)
    if f.ndim != 2 or f.shape[0] == 0:
        return -1
    return int(lib.oracle_first_dominated(f.shape[0], f.shape[1], _ptr(f, ctypes.c_int64)))


def first_uncovered(exact, apx, eps_ppm: int) -> int:
    """-1 when every row y of `exact` has a row a of `apx` with
    a <= (1 + eps_ppm / 10^6) y in every component, else the first y without."""
    lib = _load()
    e = np.ascontiguousarray(exact, dtype=np.int64)
    a = np.ascontiguousarray(apx, dtype=np.int64)
    if e.shape[0] == 0:
        return -1
    d = e.shape[1]
    a = a.reshape(-1, d)
    return int(lib.oracle_first_uncovered(e.shape[0], _ptr(e, ctypes.c_int64), a.shape[0],
                                          _ptr(a, ctypes.c_int64), d, int(eps_ppm)))

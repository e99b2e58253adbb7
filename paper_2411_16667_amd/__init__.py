"""Python binding of libmos (exact multi-objective shortest paths on MI355X).

Argument marshalling only: every step of the search runs in the HIP kernels
of ``libmos.so``; this module converts numpy arrays to C pointers and C results
back to numpy.  The function names follow the C ABI in ``include/mos.h``.
If the shared library has not been built, importing this package raises.

PyTorch plays no role in the computation.  ``use_torch_allocator()`` routes the
library's device allocations through PyTorch's caching allocator, and a torch
stream can be passed as ``stream=`` to any solve call.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmos.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mos.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2411_16667_amd/build.py` (there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

MOS_OK = 0
POP_ORDERS = {"lexicographic": 0, "generation": 1}  # mos_options.pop_order
STATUS_NAMES = ["MOS_OK", "MOS_E_INVALID_ARG", "MOS_E_NEGATIVE_COST", "MOS_E_OVERFLOW_RISK",
                "MOS_E_NO_DEVICE", "MOS_E_DEVICE", "MOS_E_OUT_OF_MEMORY", "MOS_E_LABEL_LIMIT",
                "MOS_E_CANCELLED", "MOS_E_NOT_READY", "MOS_E_STEP_LIMIT"]
for _i, _n in enumerate(STATUS_NAMES):
    globals()[_n] = _i


class mos_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_objectives", ctypes.c_int32),
                ("batch_width", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("label_limit", ctypes.c_int64), ("mem_budget", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("costs_only", ctypes.c_int32),
                ("steps_per_poll", ctypes.c_int32), ("profile_kernels", ctypes.c_int32),
                ("heuristic_radius", ctypes.c_int32), ("step_budget", ctypes.c_int64),
                ("pop_order", ctypes.c_int32), ("epsilon_ppm", ctypes.c_int32),
                ("eager_goal", ctypes.c_int32), ("pipelined", ctypes.c_int32),
                ("persistent_query", ctypes.c_int32)]


class mos_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("pops", "goal_pops", "candidates", "p_pairs", "group_pairs", "frontier_pairs",
                 "inserted", "pruned", "steps", "front", "frontier_bytes", "killed",
                 "frontier_bytes_onepass", "pairs_onepass", "near_scanned", "far_scanned",
                 "tie_entries", "front_reads")] + \
               [("search_ms", ctypes.c_double), ("heuristic_ms", ctypes.c_double),
                ("open_min_f1", ctypes.c_int64)]


_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "mos_graph_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _i64p,
                                        _i32p, _i32p, ctypes.POINTER(_vp)]),
    "mos_graph_destroy": (None, [_vp]),
    "mos_solve": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(mos_options), ctypes.POINTER(_vp)]),
    "mos_solve_batch": (ctypes.c_int, [_vp, ctypes.c_int32, _i32p, _i32p, _i32p,
                                       ctypes.POINTER(mos_options), ctypes.POINTER(_vp), _i32p]),
    "mos_solve_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(mos_options), _i32p, ctypes.c_int64,
                                         _i64p, ctypes.POINTER(mos_stats)]),
    "mos_result_size": (ctypes.c_int64, [_vp]),
    "mos_result_dim": (ctypes.c_int32, [_vp]),
    "mos_result_costs": (ctypes.c_int, [_vp, _i32p]),
    "mos_result_path": (ctypes.c_int, [_vp, ctypes.c_int64, _i32p, ctypes.c_int64, _i64p]),
    "mos_result_stats": (ctypes.c_int, [_vp, ctypes.POINTER(mos_stats)]),
    "mos_result_destroy": (None, [_vp]),
    "mos_set_allocator": (ctypes.c_int, [_ALLOC_FN, _FREE_FN, _vp]),
    "mos_server_create": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "mos_server_create_ex": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.POINTER(mos_options), ctypes.POINTER(_vp)]),
    "mos_server_submit": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "mos_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "mos_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(_vp)]),
    "mos_server_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "mos_server_counters": (ctypes.c_int, [_vp, _i64p]),
    "mos_server_destroy": (None, [_vp]),
    "mos_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mos_last_error": (ctypes.c_char_p, []),
    "mos_heuristic": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _i32p]),
    "mos_session_create": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(mos_options), ctypes.POINTER(_vp)]),
    "mos_session_step": (ctypes.c_int, [_vp, ctypes.c_int64, _i32p]),
    "mos_session_stats": (ctypes.c_int, [_vp, ctypes.POINTER(mos_stats)]),
    "mos_session_result": (ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    "mos_session_kernel_count": (ctypes.c_int32, []),
    "mos_session_set_profile": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "mos_session_kernel_times": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_char_p),
                                                ctypes.POINTER(ctypes.c_double), _i64p]),
    "mos_session_launch_counts": (ctypes.c_int, [_vp, _i64p, _i64p, _i64p]),
    "mos_session_front": (ctypes.c_int, [_vp, _i32p, ctypes.POINTER(_vp)]),
    "mos_session_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

raw = _lib  # the C functions, for tests that drive the ABI directly


class MosError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = _lib.mos_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}"
                         f" ({msg})")


def _check(st: int, where: str):
    if st != MOS_OK:
        raise MosError(st, where)


def exported_symbols_in_header() -> list:
    """Function names declared in include/mos.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mos_[a-z_0-9]+)\s*\(", txt)))


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


# --------------------------------------------------------------------- graph
class Graph:
    """A device-resident graph (``mos_graph_create``)."""

    def __init__(self, n, row_ptr, col, cost):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        cost = np.asarray(cost)
        if cost.ndim == 1:
            cost = cost[:, None]
        self.cost = np.ascontiguousarray(cost, dtype=np.int32)
        self.D = int(self.cost.shape[1])
        h = _vp()
        st = _lib.mos_graph_create(self.n, int(self.col.shape[0]), self.D,
                                   _p(self.row_ptr, ctypes.c_int64), _p(self.col, ctypes.c_int32),
                                   _p(self.cost, ctypes.c_int32), ctypes.byref(h))
        _check(st, "mos_graph_create")
        self._h = h

    @classmethod
    def from_gen(cls, g):
        return cls(g.n, g.row_ptr, g.col, g.cost)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.mos_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mos_graph_create(n, row_ptr, col, cost) -> Graph:
    return Graph(n, row_ptr, col, cost)


# -------------------------------------------------------------------- result
@dataclasses.dataclass
class Result:
    costs: np.ndarray      # int32[size, d], lexicographically ascending
    paths: list | None     # int32 arc-id arrays, or None (costs only)
    stats: dict
    # False for a step-limited or so-far result: costs are then exactly the
    # front's entries whose first objective is below stats["open_min_f1"]
    complete: bool = True


def _take_result(h, complete: bool = True) -> Result:
    try:
        n = _lib.mos_result_size(h)
        d = _lib.mos_result_dim(h)
        costs = np.zeros((n, d), dtype=np.int32)
        if n:
            _check(_lib.mos_result_costs(h, _p(costs, ctypes.c_int32)), "mos_result_costs")
        paths = []
        ln = ctypes.c_int64()
        for i in range(n):
            st = _lib.mos_result_path(h, i, None, 0, ctypes.byref(ln))
            if st != MOS_OK:
                paths = None
                break
            p = np.zeros(ln.value, dtype=np.int32)
            if ln.value:
                _check(_lib.mos_result_path(h, i, _p(p, ctypes.c_int32), ln.value, ctypes.byref(ln)),
                       "mos_result_path")
            paths.append(p)
        s = mos_stats()
        _check(_lib.mos_result_stats(h, ctypes.byref(s)), "mos_result_stats")
        stats = {f: getattr(s, f) for f, _ in mos_stats._fields_}
    finally:
        _lib.mos_result_destroy(h)
    return Result(costs, paths, stats, complete)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_options(n_objectives=0, batch_width=0, max_slots=0, label_limit=0, mem_budget=0,
                 stream=None, costs_only=False, steps_per_poll=0,
                 profile_kernels=False, heuristic_radius=0, step_budget=0,
                 pop_order="lexicographic", epsilon_ppm=0, eager_goal=False,
                 pipelined=False, persistent_query=False) -> mos_options:
    o = mos_options()
    o.struct_size = ctypes.sizeof(mos_options)
    o.n_objectives = int(n_objectives)
    o.batch_width = int(batch_width)
    o.max_slots = int(max_slots)
    o.label_limit = int(label_limit)
    o.mem_budget = int(mem_budget)
    o.stream = _stream_ptr(stream)
    o.costs_only = 1 if costs_only else 0
    o.steps_per_poll = int(steps_per_poll)
    # True = every kernel of the step; an int = bit mask over the step's kernels
    o.profile_kernels = -1 if profile_kernels is True else int(profile_kernels)
    o.heuristic_radius = int(heuristic_radius)
    o.step_budget = int(step_budget)
    o.pop_order = POP_ORDERS[pop_order] if isinstance(pop_order, str) else int(pop_order)
    o.epsilon_ppm = int(epsilon_ppm)
    o.eager_goal = 1 if eager_goal else 0
    o.pipelined = 1 if pipelined else 0
    o.persistent_query = 1 if persistent_query else 0
    return o


def mos_solve(graph: Graph, start: int, goal: int, **opts) -> Result:
    """The exact front; with step_budget, a query still running after that many
    steps returns its exact prefix (Result.complete False)."""
    o = make_options(**opts)
    h = _vp()
    st = _lib.mos_solve(graph.handle, int(start), int(goal), ctypes.byref(o), ctypes.byref(h))
    if st == MOS_E_STEP_LIMIT and h:
        return _take_result(h, complete=False)
    _check(st, "mos_solve")
    return _take_result(h)


def mos_solve_noalloc(graph: Graph, start: int, goal: int, cap: int = 1 << 16, **opts) -> Result:
    """Costs-only solve with no device allocation (``mos_solve_noalloc``);
    `cap` bounds the front size the output buffer holds."""
    o = make_options(**opts)
    d = graph.D if o.n_objectives == 0 else o.n_objectives
    buf = np.zeros((max(int(cap), 1), d), dtype=np.int32)
    n = ctypes.c_int64()
    s = mos_stats()
    _check(_lib.mos_solve_noalloc(graph.handle, int(start), int(goal), ctypes.byref(o),
                                  _p(buf, ctypes.c_int32), int(cap), ctypes.byref(n),
                                  ctypes.byref(s)), "mos_solve_noalloc")
    stats = {f: getattr(s, f) for f, _ in mos_stats._fields_}
    return Result(buf[:n.value].copy(), None, stats)


def mos_solve_batch(graph: Graph, starts, goals, n_objectives=None, **opts):
    """Returns a list of (status, Result or None), one per query."""
    starts = np.ascontiguousarray(starts, dtype=np.int32)
    goals = np.ascontiguousarray(goals, dtype=np.int32)
    nq = int(starts.shape[0])
    nobj = None if n_objectives is None else np.ascontiguousarray(n_objectives, dtype=np.int32)
    o = make_options(**opts)
    outs = (_vp * max(nq, 1))()
    sts = np.zeros(max(nq, 1), dtype=np.int32)
    rc = _lib.mos_solve_batch(graph.handle, nq, _p(starts, ctypes.c_int32),
                              _p(goals, ctypes.c_int32),
                              None if nobj is None else _p(nobj, ctypes.c_int32),
                              ctypes.byref(o), outs, _p(sts, ctypes.c_int32))
    if rc not in (MOS_OK,) and not np.any(sts[:nq] != MOS_E_NOT_READY):
        raise MosError(rc, "mos_solve_batch")
    res = []
    for i in range(nq):
        st = int(sts[i])
        res.append((st, _take_result(outs[i], complete=st == MOS_OK) if outs[i] else None))
    return res


def mos_heuristic(graph: Graph, goal: int, n_objectives: int = 0) -> np.ndarray:
    d = graph.D if n_objectives == 0 else int(n_objectives)
    h = np.zeros((d, graph.n), dtype=np.int32)
    _check(_lib.mos_heuristic(graph.handle, int(goal), int(n_objectives), _p(h, ctypes.c_int32)),
           "mos_heuristic")
    return h


# ------------------------------------------------------------------- session
class Session:
    """One query stepped on demand (``mos_session_*``)."""

    def __init__(self, graph: Graph, start: int, goal: int, **opts):
        self.graph = graph
        o = make_options(**opts)
        h = _vp()
        _check(_lib.mos_session_create(graph.handle, int(start), int(goal), ctypes.byref(o),
                                       ctypes.byref(h)), "mos_session_create")
        self._h = h

    def step(self, nsteps: int) -> bool:
        done = ctypes.c_int32()
        _check(_lib.mos_session_step(self._h, int(nsteps), ctypes.byref(done)), "mos_session_step")
        return bool(done.value)

    def stats(self) -> dict:
        s = mos_stats()
        _check(_lib.mos_session_stats(self._h, ctypes.byref(s)), "mos_session_stats")
        return {f: getattr(s, f) for f, _ in mos_stats._fields_}

    def result(self) -> Result:
        h = _vp()
        _check(_lib.mos_session_result(self._h, ctypes.byref(h)), "mos_session_result")
        return _take_result(h)

    def front_so_far(self):
        """(goal front so far as a Result, smallest F1 left in OPEN): the
        entries whose first objective is below that bound are final."""
        h = _vp()
        m = ctypes.c_int32()
        _check(_lib.mos_session_front(self._h, ctypes.byref(m), ctypes.byref(h)),
               "mos_session_front")
        return _take_result(h, complete=False), int(m.value)

    def set_profile(self, mask: int) -> None:
        """Time the kernels whose bit is set (kernel order of kernel_times); 0 = none."""
        _check(_lib.mos_session_set_profile(self._h, ctypes.c_int32(mask & 0xffffffff).value),
               "mos_session_set_profile")

    def kernel_names(self) -> list:
        return list(self.kernel_times().keys())

    def kernel_times(self) -> dict:
        out = {}
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        for i in range(_lib.mos_session_kernel_count()):
            _check(_lib.mos_session_kernel_times(self._h, i, ctypes.byref(name), ctypes.byref(ms),
                                                 ctypes.byref(n)), "mos_session_kernel_times")
            out[name.value.decode()] = (ms.value, n.value)
        return out

    def launch_counts(self) -> dict:
        """Graph replays (and steps per replay) and directly launched steps so far."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.mos_session_launch_counts(self._h, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.byref(c)), "mos_session_launch_counts")
        return {"graph_replays": a.value, "steps_per_replay": b.value, "direct_steps": c.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.mos_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -------------------------------------------------------------------- server
class Server:
    """Continuous-batching request loop (``mos_server_*``)."""

    def __init__(self, graph: Graph, mem_budget: int = 0, max_slots: int = 0, **opts):
        """opts: solve options applied to every query (batch_width,
        steps_per_poll, step_budget, costs_only, ...; mos_server_create_ex)."""
        self.graph = graph
        h = _vp()
        if opts:
            o = make_options(**opts)
            _check(_lib.mos_server_create_ex(graph.handle, int(mem_budget), int(max_slots),
                                             ctypes.byref(o), ctypes.byref(h)),
                   "mos_server_create_ex")
        else:
            _check(_lib.mos_server_create(graph.handle, int(mem_budget), int(max_slots),
                                          ctypes.byref(h)), "mos_server_create")
        self._h = h

    def submit(self, start, goal, n_objectives=0) -> int:
        t = ctypes.c_uint64()
        _check(_lib.mos_server_submit(self._h, int(start), int(goal), int(n_objectives),
                                      ctypes.byref(t)), "mos_server_submit")
        return t.value

    def poll(self, ticket):
        """None while not ready, else (status, Result or None); raises for an
        unknown or already collected ticket."""
        h = _vp()
        st = _lib.mos_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(h))
        if st == MOS_E_NOT_READY:
            return None
        if st == MOS_E_INVALID_ARG:
            raise MosError(st, "mos_server_poll")
        return st, (_take_result(h, complete=st == MOS_OK)
                    if st in (MOS_OK, MOS_E_STEP_LIMIT) and h else None)

    def wait(self, ticket, timeout_ms=-1):
        h = _vp()
        st = _lib.mos_server_wait(self._h, ctypes.c_uint64(ticket), int(timeout_ms), ctypes.byref(h))
        if st == MOS_E_NOT_READY:
            return None
        if st == MOS_E_INVALID_ARG:
            raise MosError(st, "mos_server_wait")
        return st, (_take_result(h, complete=st == MOS_OK)
                    if st in (MOS_OK, MOS_E_STEP_LIMIT) and h else None)

    def cancel(self, ticket):
        _check(_lib.mos_server_cancel(self._h, ctypes.c_uint64(ticket)), "mos_server_cancel")

    def counters(self) -> dict:
        a = np.zeros(6, dtype=np.int64)
        _check(_lib.mos_server_counters(self._h, _p(a, ctypes.c_int64)), "mos_server_counters")
        return dict(zip(["submitted", "finished", "resident", "queued", "ticks", "readmissions"],
                        (int(x) for x in a)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.mos_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mos_server_create(graph: Graph, mem_budget: int = 0, max_slots: int = 0) -> Server:
    return Server(graph, mem_budget, max_slots)


# ----------------------------------------------------------------- allocator
_torch_cb = None


def use_torch_allocator(enable: bool = True):
    """Route libmos device allocations through PyTorch's caching allocator."""
    global _torch_cb
    if not enable:
        _check(_lib.mos_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "mos_set_allocator")
        _torch_cb = None
        return
    import torch

    dev = torch.cuda.current_device()

    def _alloc(nbytes, stream, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0))
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    _torch_cb = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(_lib.mos_set_allocator(_torch_cb[0], _torch_cb[1], None), "mos_set_allocator")

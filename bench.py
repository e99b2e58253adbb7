"""Benchmark: dominance checks per second of the batched label step on one MI355X.

Workload: the ship-routing-shaped query (256x256 8-connected grid, d = 3
smooth-field int32 costs, start and goal at opposite corners).  Its exact
front is far too large for a run of a few minutes (hundreds of thousands of
Pareto-optimal costs), so a bench "step" is one batched label step of that
search (every stage of the hot path over one batch of B popped labels): W
untimed warm-up steps, then K timed steps, with the query's state resident on
the device throughout.  The value is dominance pair checks per second: every
(candidate, stored vector) comparison the method makes against the goal front,
against same-step candidates of the same node, and against node frontiers.

Prints one JSON line.  The search is first taken --depth-steps deep (always,
whatever --warmup is); a per-kernel table at that depth picks the dominant
kernel; the timed steps then replay the captured step graph as mos_solve
does, pipelined (the next batch popped beside the current batch's goal-front
filter; --synchronous for the plain order).  Also reports the roofline of the dominant kernel (its durations from
HIP events in an event window of the same length right after the timed
steps, its algorithmic bytes from the search counters of that window, its
measured HBM traffic from the committed PMC summary when that summary
matches the current kernel sources), the CPU oracle's check rate on a
bounded sample of the same query, and queries/s of one batched call against
a loop of single solves on short-range queries of the same grid.

`--workload served` instead runs the request loop on the 1M-node road-like
graph (saturation and Poisson arrivals, p50/p99 latency) and prints its own
JSON line; `--workload routes` solves the five time-expanded ship routes
shaped like the paper's Table 2 at that table's largest objective counts (up
to 12), whole queries, and prints its own JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# int32 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane operations/s
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
METRIC = "dominance checks/s + queries/s (batched vs plain), exact Pareto front, 1 GPU"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed label steps")
    ap.add_argument("--warmup", type=int, default=16,
                    help="untimed label steps right before the timed ones, launched the same "
                         "way (after the depth steps and the per-kernel table)")
    ap.add_argument("--depth-steps", type=int, default=480,
                    help="label steps run first, always, to take the search to the depth where "
                         "the timed steps start (480 steps of B = 32768 reach about 16M "
                         "labels; frontiers and the goal front are then near their "
                         "steady-state sizes)")
    ap.add_argument("--batch-width", type=int, default=32768,
                    help="labels popped per step (the widest batch the library takes; at this "
                         "depth 16384 gives 21.8M pops/s and 32768 about 25M)")
    ap.add_argument("--profile-steps", type=int, default=32,
                    help="steps after the depth steps with every kernel timed (per-kernel "
                         "table at depth; picks the dominant kernel)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="length of the oracle sample for the CPU baseline (0 = skip)")
    ap.add_argument("--time-to-front", type=int, default=1,
                    help="1 = also time whole queries with stored oracle fronts to the exact "
                         "front (routes at Table 2's objective counts, mid-range ship-grid "
                         "queries); 0 = skip")
    ap.add_argument("--queries", type=int, default=64,
                    help="queries of the batched-vs-plain comparison (0 = skip)")
    ap.add_argument("--qdist", type=int, nargs=2, default=(10, 60),
                    help="Manhattan distance range of those queries")
    ap.add_argument("--query-width", type=int, default=0,
                    help="batch width B of every query in that comparison (0 = picked by "
                         "the autotuner on a sample of the queries)")
    ap.add_argument("--workload", choices=("steps", "served", "routes", "orders", "pipelined",
                                           "c4"),
                    default="steps",
                    help="steps: label steps of the ship-routing query (the headline line); "
                         "served: the request loop on the 1M-node road-like graph; "
                         "routes: whole queries on the time-expanded routes at up to 12 "
                         "objectives; orders: lexicographic against generation (FIFO) "
                         "OPEN order, labels popped and time to the exact front; "
                         "pipelined: synchronous against pipelined steps, the same measures; "
                         "c4: the 512 uneven queries of the batched configuration in one "
                         "batched call under a step budget, against the plain path on a sample")
    ap.add_argument("--c4-budget", type=int, default=256,
                    help="c4 workload: steps per query (a query still running returns the "
                         "exact part of its front)")
    ap.add_argument("--c4-width", type=int, default=1024, help="c4 workload: batch width")
    ap.add_argument("--persistent-query", action="store_true",
                    help="queries leg and served workload: every query runs its steps in "
                         "one workgroup of its own (mos_options.persistent_query), against "
                         "the default multi-kernel step")
    ap.add_argument("--synchronous", action="store_true",
                    help="steps workload: run the label steps synchronously (default: "
                         "pipelined, the next batch extracted beside the current batch's "
                         "goal-front filter; 1.07 against 1.12 ms per step at this depth)")
    ap.add_argument("--route-width", type=int, default=0,
                    help="routes workload: batch width B (0 = picked per route by the "
                         "autotuner from 1024, 4096, 16384; the routes at 32768 are kept off "
                         "the GPU until an unexplained fault is understood)")
    ap.add_argument("--route-repeats", type=int, default=3,
                    help="routes workload: timed solves per route (the median is reported)")
    ap.add_argument("--route-sweep", type=int, nargs="*", default=None, metavar="B",
                    help="routes workload: also solve routes 1 and 5 at these batch widths and "
                         "report labels popped against the oracle's (work efficiency)")
    ap.add_argument("--served-queries", type=int, default=600,
                    help="queries per arrival-rate point of the served workload")
    ap.add_argument("--radius", type=float, default=0.02,
                    help="served workload: goals within this distance of the start")
    ap.add_argument("--slots", type=int, default=64, help="served workload: resident queries")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 4 times (a kernel of known "
                         "HBM traffic, to scale hardware byte counters) and exit")
    return ap.parse_args()


# Algorithmic bytes of each step kernel: what its part of the step has to move
# through HBM at least, from the search counters (deltas over the timed steps).
# d objectives; int32 words; label state 1 byte.
def kernel_bytes(name, c, d, steps):
    pops = c["pops"] + c["killed"]          # labels taken from OPEN
    cands, acc = c["candidates"], c["inserted"]
    fb, fb1 = c["frontier_bytes"], c["frontier_bytes_onepass"]
    return {
        "k_far_hist": 9 * c["far_scanned"],                 # F1, label id, state
        "k_far_move": 17 * c["far_scanned"],                # + the entry written back
        "k_open_hist": 9 * c["near_scanned"],
        "k_open_threshold": 8 * 4096 * steps,               # histogram read + reset
        "k_open_scatter": 17 * c["near_scanned"],
        "k_batch_finalize": 28 * pops + (8 + 8 * d + 4) * c["tie_entries"],
        # per batch label: id, node and (regular ones) two row offsets; per tie
        # entry: state, label, F1.  The scan reads the same again and writes
        # reg/reg_off/reg_kill or goal_lab/goal flag, and an entry sent back
        # to OPEN (F1, label; every tie entry counted: an upper bound)
        "k_split_count": 24 * pops - 16 * c["goal_pops"] + 12 * c["tie_entries"],
        "k_split_scan": 36 * pops - 20 * c["goal_pops"] + 20 * c["tie_entries"],
        "k_goal_pairs": 4 * d * c["front_reads"] + 4 * d * c["goal_pops"],
        "k_goal_merge": (8 + 8 * d) * c["goal_pops"],
        "k_popcheck": (8 + 8 * d) * pops,
        "k_expand": (16 + 12 * d) * cands,
        "k_pfilter": (4 + 8 * d) * acc,                     # labels inserted this step
        "k_group_count": 8 * cands,
        "k_group_offsets": 12 * cands,
        "k_group_scatter": 12 * cands,
        "k_group_process": fb1,
        # the large groups' pair tiles, both passes together (PAIR_PASSES):
        # each frontier entry read once
        "k_group_pairs": fb - fb1,
        "k_group_pairs2": fb - fb1,
        "k_group_finish": fb - fb1,
        "k_accept_count": 4 * cands,
        "k_accept_scan": 4 * cands + 12 * acc,
        "k_insert": (12 * d + 24) * acc,
        "k_step_end": 0,
    }.get(name, 0)


# The large groups' pair tiles run as two launches of one kernel: the first
# pass (candidates against candidates and against each group's first frontier
# tile) and the second (the other frontier tiles, candidates already rejected
# skipped).  Their roofline takes both launches as one unit.
PAIR_PASSES = ("k_group_pairs", "k_group_pairs2")
PAIR_UNIT = "k_group_pairs+k_group_pairs2"


def kernel_ops(name, c, d):
    """int32 VALU comparisons the kernel's dominance tests need (0: none)."""
    if name == "k_group_process":
        return 2 * d * c["pairs_onepass"]   # <= both ways per candidate pair
    if name in ("k_group_pairs", PAIR_UNIT):
        # the large groups' pairs, both passes together: every (candidate,
        # frontier entry) and (candidate, candidate) pair the method decides;
        # the second pass skips the rows of candidates the first one rejected
        return 2 * d * (c["frontier_pairs"] + c["group_pairs"] - c["pairs_onepass"])
    if name in ("k_pfilter", "k_popcheck", "k_goal_pairs"):
        return d * c["p_pairs"]
    return 0


KERNEL_SOURCES = ("paper_2411_16667_amd/csrc/step.hip", "paper_2411_16667_amd/csrc/mos_core.h",
                  "paper_2411_16667_amd/csrc/kernels.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_ship256_steps.md")


def kernel_source_digest() -> str:
    """sha256/16 of the kernel sources with // comments and blank lines
    removed: it changes with the code the counters were taken on, not with
    an edit of a comment."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            lines = (line.split("//", 1)[0].rstrip() for line in fh)
            h.update("\n".join(x for x in lines if x).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, batch_width):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    when there is none for this kernel and batch width or the kernel sources
    have changed since the counters were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    meta = dict(line[2:].split(": ", 1) for line in text.splitlines()
                if line.startswith("- ") and ": " in line)
    if (meta.get("kernel sources sha256/16") or " ").split()[0] != kernel_source_digest():
        return None
    if meta.get("batch width") != str(batch_width):
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and cells[0] == kernel:
            try:
                return float(cells[3])
            except ValueError:
                return None
    return None


def cpu_baseline(g, s, t, seconds):
    import oracle

    r = oracle.solve(g, s, t, 3, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN, time_limit=seconds)
    st = r.stats
    pairs = st["frontier_pairs"] + st["p_pairs"]
    secs = max(st["search_seconds"], 1e-9)
    return {"value": pairs / secs, "unit": "checks/s", "cores": 1, "kind": "oracle",
            "sample": f"first {secs:.1f} s of the sequential search of the same query "
                      f"({st['pops']} labels processed, {pairs} pair checks)"}


def cpu_all_cores(g, S, T, seconds):
    """The oracle as a pool of one query per host core (threads: the oracle
    releases the interpreter while it searches) over the same start/goal list
    as the batched-vs-plain comparison, cycling through it until about
    `seconds` have passed; queries/s with the core count used."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))  # the machine's CPU share for one GPU
    oracle.build()
    flags = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN
    stop = time.perf_counter() + seconds

    def worker(w):
        n, i = 0, w
        while time.perf_counter() < stop:
            q = i % len(S)
            r = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=flags, want_paths=False)
            assert r.status == "ok"
            n += 1
            i += cores
        return n

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        done = sum(ex.map(worker, range(cores)))
    wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} solves of the {len(S)} batched-comparison queries in {wall:.1f} s, "
                      f"one query per core"}


def time_to_front(mos, gen):
    """Whole queries with stored oracle fronts (the five time-expanded routes
    at Table 2's objective counts, the mid-range ship-grid queries): wall time
    of mos_solve to the exact front (median of three after an untimed one),
    checked against the stored front, with the oracle's own pair checks for
    the same query (recorded when it was stored) over that time: checks/s in
    the oracle's units."""
    import glob

    import numpy as np

    work = []
    for r in sorted(gen.ROUTE_SHAPES):
        g, s, t = gen.tmplar_route(r, 12, 0)
        work.append((g, s, t, gen.ROUTE_MAX_OBJECTIVES[r], 16384,
                     os.path.join(ROOT, "tests", "golden", "routes", f"r{r}.txt.gz")))
    ship = gen.ship_grid(256, 256, 3, 0)
    for f in sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "c4mid", "q*.txt.gz"))):
        h, _ = _stored(f)
        work.append((ship, int(h["start"]), int(h["goal"]), 3, 4096, f))
    rows, graphs = [], {}
    for g, s, t, d, B, ref in work:
        G = graphs.setdefault(id(g), mos.Graph.from_gen(g))
        hdr, want = _stored(ref)
        kw = dict(n_objectives=d, batch_width=B)
        res = mos.mos_solve(G, s, t, **kw)
        walls = []
        for _ in range(3):
            t0 = time.perf_counter()
            res = mos.mos_solve(G, s, t, **kw)
            walls.append(time.perf_counter() - t0)
        wall = float(np.median(walls))
        row = {"workload": hdr["workload"], "d": d, "batch_width": B, "front": int(want.shape[0]),
               "seconds": wall, "same_front_as_stored_oracle":
                   bool(np.array_equal(res.costs.astype(np.int64), want)),
               "oracle_seconds_when_stored": float(hdr["search_seconds"])}
        if "pairs" in hdr:
            row["oracle_pairs"] = int(hdr["pairs"])
            row["oracle_equivalent_checks_per_s"] = int(hdr["pairs"]) / wall
        rows.append(row)
    with_pairs = [r for r in rows if "oracle_pairs" in r]
    return {"queries": rows,
            "all_same_fronts": all(r["same_front_as_stored_oracle"] for r in rows),
            "seconds_total": sum(r["seconds"] for r in rows),
            "oracle_equivalent_checks_per_s":
                (sum(r["oracle_pairs"] for r in with_pairs) / sum(r["seconds"] for r in with_pairs)
                 if with_pairs else None)}


def batched_vs_plain(mos, gen, G, a):
    """Queries/s of one mos_solve_batch call against a loop of mos_solve over
    the same start/goal list on the same grid (same B, paths included; B from
    the autotuner unless --query-width is given)."""
    import numpy as np

    S, T = gen.ship_queries(256, 256, a.queries, seed=1000, dmin=a.qdist[0], dmax=a.qdist[1])
    tuned = None
    B = a.query_width
    if B == 0:
        from paper_2411_16667_amd.autotune import tune_batch_width

        tuned = tune_batch_width(G, S, T, widths=(256, 1024, 4096), sample=len(S),
                                 costs_only=False)
        B = tuned["batch_width"]
    # engines are cached per (slot count, width, ...): one untimed call of each
    # form first, so that both timed forms reuse their engine
    pq = a.persistent_query
    mos.mos_solve_batch(G, S, T, batch_width=B, persistent_query=pq)
    mos.mos_solve(G, int(S[0]), int(T[0]), batch_width=B, persistent_query=pq)
    t0 = time.perf_counter()
    res = mos.mos_solve_batch(G, S, T, batch_width=B, persistent_query=pq)
    t_batched = time.perf_counter() - t0
    t0 = time.perf_counter()
    plain = [mos.mos_solve(G, int(S[q]), int(T[q]), batch_width=B, persistent_query=pq)
             for q in range(len(S))]
    t_plain = time.perf_counter() - t0
    same = all(st == mos.MOS_OK and np.array_equal(r.costs, p.costs)
               for (st, r), p in zip(res, plain))
    fronts = [len(p.costs) for p in plain]
    return {"queries": len(S), "manhattan_distance": list(a.qdist), "batch_width": B,
            "autotune": tuned, "persistent_query": bool(pq),
            "batched_qps": len(S) / t_batched, "plain_qps": len(S) / t_plain,
            "speedup": t_plain / t_batched, "same_fronts": bool(same),
            "front_sizes": {"min": min(fronts), "median": int(np.median(fronts)), "max": max(fronts)}}


def run_stream(srv, S, T, D, arrivals):
    """Submit query i at time arrivals[i] (seconds from now); a poller thread
    collects results.  Returns (latencies in s from arrival, wall seconds, results)."""
    import threading

    n = len(S)
    tickets = [None] * n
    done_at = [None] * n
    res = [None] * n
    submitted = threading.Event()
    t0 = time.perf_counter()

    def poller():
        pending = set()
        nxt = 0
        while True:
            while nxt < n and tickets[nxt] is not None:
                pending.add(nxt)
                nxt += 1
            for i in list(pending):
                r = srv.poll(tickets[i])
                if r is not None:
                    done_at[i] = time.perf_counter()
                    res[i] = r
                    pending.discard(i)
            if submitted.is_set() and nxt == n and not pending:
                return
            time.sleep(0.0002)

    th = threading.Thread(target=poller)
    th.start()
    for i in range(n):
        delay = t0 + arrivals[i] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets[i] = srv.submit(int(S[i]), int(T[i]), int(D[i]))
    submitted.set()
    th.join()
    wall = max(done_at) - t0
    lat = [done_at[i] - (t0 + arrivals[i]) for i in range(n)]
    return lat, wall, res


def c4_bench(a):
    """The batched configuration as generated: 512 start/goal pairs on the 256x256
    ship grid with Manhattan distance uniform in [10, 400] (fronts from a few
    vectors to beyond 10^4), one mos_solve_batch call with 256 resident slots.
    The largest of these queries do not finish in a bench's time, so every
    query runs under a step budget: one still running then returns the exact
    part of its front (the entries below its OPEN bound).  The plain path
    (mos_solve one query at a time, the same budget and width) runs on the first
    64 queries; both rates count queries returned per second."""
    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    g, S, T = gen.config4(0)
    G = mos.Graph.from_gen(g)
    kw = dict(batch_width=a.c4_width, step_budget=a.c4_budget, steps_per_poll=16)
    mos.mos_solve_batch(G, S[:8], T[:8], max_slots=256, **kw)  # engine and kernels warm
    t0 = time.perf_counter()
    res = mos.mos_solve_batch(G, S, T, max_slots=256, **kw)
    tb = time.perf_counter() - t0
    complete = sum(1 for st, _ in res if st == mos.MOS_OK)
    assert all(st in (mos.MOS_OK, mos.MOS_E_STEP_LIMIT) for st, _ in res)
    vectors = sum(int(r.costs.shape[0]) for _, r in res)
    print(f"c4: batched call {tb:.1f} s, {complete} complete fronts", file=sys.stderr, flush=True)
    npl = 64
    mos.mos_solve(G, int(S[0]), int(T[0]), **kw)
    t0 = time.perf_counter()
    plain = [mos.mos_solve(G, int(S[q]), int(T[q]), **kw) for q in range(npl)]
    tp = time.perf_counter() - t0
    same = all(np.array_equal(p.costs, r.costs) for p, (_, r) in zip(plain, res[:npl]))
    fronts = [int(r.costs.shape[0]) for st, r in res if st == mos.MOS_OK]
    out = {"metric": "queries/s of the 512-query batched configuration (step-budgeted, exact "
                     "fronts or exact prefixes), batched vs plain, 1 GPU",
           "value": len(S) / tb, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "512 queries, 256x256 ship grid d=3, Manhattan distance "
                                  "U[10,400]", "batch_width": a.c4_width, "slots": 256,
                      "step_budget": a.c4_budget},
           "seconds": tb, "complete_fronts": complete, "prefixes": len(S) - complete,
           "vectors_returned": vectors,
           "complete_front_sizes": {"median": int(np.median(fronts)) if fronts else 0,
                                    "max": max(fronts) if fronts else 0},
           "plain_qps_first_64": npl / tp, "same_output_as_plain_first_64": bool(same)}
    print(json.dumps(out))


def served_bench(a):
    """The served workload: 1M-node 8-NN road-like graph, five stored objectives,
    queries with d ~ U{3,4,5} and goals within a radius of the start; one
    saturation run (all queries submitted at once), then Poisson arrivals at
    fractions of the measured saturation rate; plus the plain path (one
    mos_solve at a time) on the same queries."""
    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    t0 = time.perf_counter()
    g, rng, comp = gen.config5_graph(0)
    nq = a.served_queries
    S, T, D = gen.local_queries(g, comp, 7 * nq, seed=0, radius=a.radius)
    G = mos.Graph.from_gen(g)
    print(f"served: graph and {7 * nq} queries ready in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    # plain: one query at a time through mos_solve
    npl = min(nq, 200)
    pq = a.persistent_query
    mos.mos_solve(G, int(S[0]), int(T[0]), n_objectives=int(D[0]), persistent_query=pq)
    tp = time.perf_counter()
    plain = [mos.mos_solve(G, int(S[i]), int(T[i]), n_objectives=int(D[i]), persistent_query=pq)
             for i in range(npl)]
    plain_qps = npl / (time.perf_counter() - tp)
    print(f"served: plain {plain_qps:.1f} q/s", file=sys.stderr, flush=True)
    srv = mos.Server(G, max_slots=a.slots, persistent_query=True) if pq else \
        mos.Server(G, max_slots=a.slots)
    lat, wall, res = run_stream(srv, S[:nq], T[:nq], D[:nq], np.zeros(nq))
    sat = nq / wall
    same = all(r is not None and r[0] == mos.MOS_OK and np.array_equal(r[1].costs, p.costs)
               for r, p in zip(res[:npl], plain))
    points = [{"rate_frac": "all at once", "offered_qps": None, "qps": sat,
               "p50_ms": 1e3 * float(np.percentile(lat, 50)),
               "p99_ms": 1e3 * float(np.percentile(lat, 99))}]
    print(f"served: saturation {sat:.1f} q/s", file=sys.stderr, flush=True)
    for k, frac in enumerate((0.1, 0.25, 0.5, 0.75, 0.9, 1.1)):
        rate = frac * sat
        lo = (k + 1) * nq
        arr = gen.poisson_arrivals(nq, rate, seed=k)
        lat, wall, res = run_stream(srv, S[lo:lo + nq], T[lo:lo + nq], D[lo:lo + nq], arr)
        ok = all(r is not None and r[0] == mos.MOS_OK for r in res)
        points.append({"rate_frac": frac, "offered_qps": rate, "qps": nq / wall,
                       "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                       "p99_ms": 1e3 * float(np.percentile(lat, 99)), "all_ok": ok})
        print(f"served: {points[-1]}", file=sys.stderr, flush=True)
    c = srv.counters()
    srv.close()
    fronts = [len(p.costs) for p in plain]
    out = {"metric": "served queries/s with p50/p99 latency (Poisson arrivals), exact Pareto "
                     "front, 1 GPU",
           "value": sat, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"1M-node 8-NN geometric graph, 5 stored objectives, d~U{{3,4,5}}, "
                                  f"goals within {a.radius} of the start", "slots": a.slots,
                      "batch_width": 256, "queries_per_point": nq,
                      "persistent_query": bool(pq)},
           "plain_qps": plain_qps, "served_vs_plain": sat / plain_qps,
           "same_fronts_as_plain": bool(same), "points": points, "server_counters": c,
           "front_sizes": {"min": min(fronts), "median": int(np.median(fronts)),
                           "max": max(fronts)}}
    print(json.dumps(out))


def routes_bench(a):
    """Whole queries on the five time-expanded routes (Table 2 shapes), each at
    Table 2's largest objective count for that route and at the batch width
    the autotuner picks for it: one untimed solve, then the median of
    --route-repeats timed solves (wall clock around mos_solve: heuristic,
    search, harvest and paths).  The CPU baseline is the oracle on
    the smallest route (whole query) and on a bounded sample of route 1."""
    import gzip

    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    rows, tot_pairs, tot_s = [], 0, 0.0
    for r in sorted(gen.ROUTE_SHAPES):
        d = gen.ROUTE_MAX_OBJECTIVES[r]
        g, s, t = gen.tmplar_route(r, 12, 0)
        G = mos.Graph.from_gen(g)
        B = a.route_width
        if B == 0:
            from paper_2411_16667_amd.autotune import tune_batch_width

            B = tune_batch_width(G, [s], [t], n_objectives=[d], widths=(1024, 4096, 16384),
                                 sample=1, costs_only=False)["batch_width"]
        kw = dict(n_objectives=d, batch_width=B)
        res = mos.mos_solve(G, s, t, **kw)
        walls = []
        for _ in range(a.route_repeats):
            t0 = time.perf_counter()
            res = mos.mos_solve(G, s, t, **kw)
            walls.append(time.perf_counter() - t0)
        wall = float(np.median(walls))
        st = res.stats
        pairs = st["p_pairs"] + st["group_pairs"] + st["frontier_pairs"]
        row = {"route": r, "nodes": g.n, "arcs": g.n_arcs, "d": d, "batch_width": B,
               "front": len(res.costs),
               "seconds": wall, "search_ms": st["search_ms"], "heuristic_ms": st["heuristic_ms"],
               "pops": st["pops"], "steps": st["steps"], "pairs": pairs, "checks_per_s": pairs / wall}
        # the stored oracle front of this route, when there is one (tests/golden/routes)
        ref = os.path.join(ROOT, "tests", "golden", "routes", f"r{r}.txt.gz")
        if os.path.exists(ref):
            hdr, rows_ref = {}, []
            with gzip.open(ref, "rt") as f:
                for line in f:
                    if line.startswith("#"):
                        k, _, v = line[1:].partition(":")
                        hdr[k.strip()] = v.strip()
                    elif line.strip():
                        rows_ref.append([int(x) for x in line.split()])
            row["same_front_as_stored_oracle"] = bool(
                hdr.get("graph_sha256_16") == g.digest()
                and np.array_equal(res.costs.astype(np.int64), np.array(rows_ref, np.int64).reshape(-1, d)))
            row["oracle_pops"] = int(hdr["pops"])
            row["oracle_seconds_when_stored"] = float(hdr["search_seconds"])
        rows.append(row)
        tot_pairs += pairs
        tot_s += wall
        print(f"routes: {row}", file=sys.stderr, flush=True)
    out = {"metric": "dominance checks/s, whole queries, exact Pareto front, 1 GPU",
           "value": tot_pairs / tot_s, "unit": "checks/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "five time-expanded ship routes shaped like Table 2 "
                                  "(10 time windows per cell), each at Table 2's largest "
                                  "objective count (12, 4, 12, 12, 6)",
                      "batch_width": a.route_width or "autotuned per route",
                      "repeats": a.route_repeats},
           "seconds_all_routes": tot_s, "routes": rows}
    if a.route_sweep:
        # labels popped per batch width against the sequential oracle's pops
        # (the paper's work-efficiency measure for its multi-pop), and time
        sweep = []
        for r in (1, 5):
            d = gen.ROUTE_MAX_OBJECTIVES[r]
            g, s, t = gen.tmplar_route(r, 12, 0)
            G = mos.Graph.from_gen(g)
            ref = next((x for x in rows if x["route"] == r), {})
            for B in a.route_sweep:
                mos.mos_solve(G, s, t, n_objectives=d, batch_width=B, costs_only=True)
                t0 = time.perf_counter()
                res = mos.mos_solve(G, s, t, n_objectives=d, batch_width=B, costs_only=True)
                wall = time.perf_counter() - t0
                pt = {"route": r, "d": d, "batch_width": B, "seconds": wall,
                      "steps": res.stats["steps"], "pops": res.stats["pops"], "front": len(res.costs)}
                if "oracle_pops" in ref:
                    pt["pops_vs_oracle"] = res.stats["pops"] / ref["oracle_pops"]
                sweep.append(pt)
                print(f"routes sweep: {pt}", file=sys.stderr, flush=True)
        out["batch_width_sweep"] = sweep
    if a.cpu_seconds > 0:
        import oracle

        flags = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN
        base = []
        for r, limit in ((4, a.cpu_seconds), (1, a.cpu_seconds)):
            d = gen.ROUTE_MAX_OBJECTIVES[r]
            g, s, t = gen.tmplar_route(r, 12, 0)
            o = oracle.solve(g, s, t, d, flags=flags, time_limit=limit)
            so = o.stats
            pairs = so["frontier_pairs"] + so["p_pairs"]
            base.append((r, o.status, so["search_seconds"], so["pops"], pairs))
        pairs = sum(b[4] for b in base)
        secs = max(sum(b[2] for b in base), 1e-9)
        out["cpu_baseline"] = {
            "value": pairs / secs, "unit": "checks/s", "cores": 1, "kind": "oracle",
            "sample": "; ".join(f"route {r}: {'whole query' if stt == 'ok' else 'first'} "
                                f"{sec:.1f} s, {pops} labels, {pr} pair checks"
                                for r, stt, sec, pops, pr in base)}
        r4 = next(b for b in base if b[0] == 4)
        if r4[1] == "ok":
            out["route4_speedup_vs_oracle"] = r4[2] / next(x for x in rows if x["route"] == 4)["seconds"]
    print(json.dumps(out))


def _stored(path):
    import importlib.util

    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(ROOT, "tests", "golden", "make_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m.read_front(path)


def compare_bench(a, study):
    """Two ways of running the same whole queries with stored oracle fronts (the
    five time-expanded routes at Table 2's objective counts, the mid-range
    ship-grid queries), at one batch width, costs only: labels popped against
    the sequential oracle's pops, steps, and wall time to the exact front
    (median of --route-repeats solves after an untimed one).
    study "orders": lexicographic priority order against the relaxed
    generation (FIFO) order of OPEN, as the paper's Section 7.1 compares a
    priority queue with a FIFO queue; the generation order runs under a step
    cap of cap_factor times the lexicographic steps.
    study "pipelined": synchronous steps against pipelined ones (the next
    batch extracted beside the current batch's goal-front filter, Section
    5.1's current and next bags)."""
    import glob

    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    if study == "orders":
        variants = [("lexicographic", dict(pop_order="lexicographic")),
                    ("generation", dict(pop_order="generation"))]
        metric = "time to the exact front, lexicographic vs generation (FIFO) OPEN order, 1 GPU"
    else:
        variants = [("synchronous", {}), ("pipelined", dict(pipelined=True))]
        metric = "time to the exact front, synchronous vs pipelined steps, 1 GPU"
    (n0, _), (n1, _) = variants
    work = []
    for r in sorted(gen.ROUTE_SHAPES):
        g, s, t = gen.tmplar_route(r, 12, 0)
        work.append((f"route{r}", g, s, t, gen.ROUTE_MAX_OBJECTIVES[r],
                     os.path.join(ROOT, "tests", "golden", "routes", f"r{r}.txt.gz")))
    ship = gen.ship_grid(256, 256, 3, 0)
    for f in sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "c4mid", "q*.txt.gz"))):
        h, _ = _stored(f)
        work.append((h["workload"], ship, int(h["start"]), int(h["goal"]), 3, f))
    B = a.route_width or 4096
    cap_factor = 32
    rows = []
    graphs = {}
    for name, g, s, t, d, ref in work:
        G = graphs.setdefault(id(g), mos.Graph.from_gen(g))
        hdr, want = _stored(ref)
        row = {"workload": name, "d": d, "batch_width": B, "oracle_pops": int(hdr["pops"]),
               "front": int(want.shape[0])}
        budget = 0
        for vname, extra in variants:
            # the second variant of the orders study gets a step cap of
            # cap_factor times the steps the first needed; a run stopped there
            # reports its exact prefix
            kw = dict(n_objectives=d, batch_width=B, costs_only=True, step_budget=budget, **extra)
            walls = []
            res = None
            try:
                for rep in range(a.route_repeats + 1):
                    t0 = time.perf_counter()
                    res = mos.mos_solve(G, s, t, **kw)
                    if rep:
                        walls.append(time.perf_counter() - t0)
                    if not res.complete:
                        walls.append(time.perf_counter() - t0)
                        break
            except mos.MosError as e:
                row[vname] = {"finished": False, "error": str(e)}
                continue
            out = {"seconds": float(np.median(walls)), "pops": res.stats["pops"],
                   "steps": res.stats["steps"], "finished": bool(res.complete),
                   "pops_vs_oracle": res.stats["pops"] / int(hdr["pops"])}
            if res.complete:
                out["same_front_as_stored_oracle"] = bool(
                    np.array_equal(res.costs.astype(np.int64), want))
            else:
                out["step_cap"] = budget
                out["exact_prefix_rows"] = int(res.costs.shape[0])
            row[vname] = out
            if study == "orders" and vname == n0:
                budget = cap_factor * max(int(res.stats["steps"]), 1)
        both = all(row[v].get("finished") for v, _ in variants)
        if both:
            row[f"{n1}_vs_{n0}_time"] = row[n1]["seconds"] / row[n0]["seconds"]
        rows.append(row)
        print(f"{study}: {row}", file=sys.stderr, flush=True)
    fin = [r for r in rows if f"{n1}_vs_{n0}_time" in r]
    t0_ = sum(r[n0]["seconds"] for r in fin)
    t1_ = sum(r[n1]["seconds"] for r in fin)
    out = {"metric": metric, "value": t1_ / t0_ if t0_ > 0 else None,
           "unit": f"time ratio {n1}/{n0}", "higher_is_better": False, "n_gpus": 1,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "time-expanded routes 1-5 at Table 2's objective counts and the "
                                  "mid-range ship-grid queries with stored oracle fronts",
                      "batch_width": B, "repeats": a.route_repeats},
           "value_over": f"{len(fin)} of {len(rows)} queries that both finished",
           f"seconds_{n0}": t0_, f"seconds_{n1}": t1_, "queries": rows}
    if study == "orders":
        out["config"]["generation_step_cap"] = f"{cap_factor}x the lexicographic steps"
        out["generation_unfinished"] = [r["workload"] for r in rows
                                        if not r["generation"].get("finished")]
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); queries are "
              "independent, so several GPUs run one server process each, with the graph "
              "replicated and no exchange between them", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    if a.workload == "served":
        served_bench(a)
        return
    if a.workload == "routes":
        routes_bench(a)
        return
    if a.workload in ("orders", "pipelined"):
        compare_bench(a, a.workload)
        return
    if a.workload == "c4":
        c4_bench(a)
        return
    if a.copy_calibration > 0:
        import torch

        n = a.copy_calibration << 18  # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n,
                          "dispatches": 4}))
        return

    g, s, t = gen.config2(0)
    G = mos.Graph.from_gen(g)
    d = 3
    # steps per captured graph: a divisor of the timed step count, so that every
    # timed step is replayed from the captured graph (the form mos_solve uses)
    K = next(k for k in range(min(32, a.steps), 0, -1) if a.steps % k == 0)
    sess = mos.Session(G, s, t, batch_width=a.batch_width, steps_per_poll=K,
                       pipelined=not a.synchronous)
    left = a.depth_steps
    while left > 0:  # in chunks, with a progress line each
        n = min(left, 256)
        sess.step(n)
        left -= n
        print(f"bench: depth, {a.depth_steps - left} steps", file=sys.stderr, flush=True)
    # per-kernel table at depth: every kernel bracketed by HIP events (the
    # kernels then launch one by one); the largest share is the dominant kernel
    pre = max(K, a.profile_steps)
    sess.set_profile(-1)
    p0 = sess.kernel_times()
    sess.step(pre)
    p1 = sess.kernel_times()
    table = {n: (p1[n][0] - p0[n][0], p1[n][1] - p0[n][1]) for n in p1}
    units = {n: v[0] for n, v in table.items() if n not in PAIR_PASSES}
    units[PAIR_UNIT] = sum(table[n][0] for n in PAIR_PASSES)
    dom = max(units, key=units.get)
    members = PAIR_PASSES if dom == PAIR_UNIT else (dom,)
    sess.set_profile(0)
    # warm-up and timed steps: replays of the captured step graph (the launch
    # form mos_solve uses), no events
    if a.warmup > 0:
        sess.step(a.warmup)
    s0, l0 = sess.stats(), sess.launch_counts()
    t0 = time.perf_counter()
    done = sess.step(a.steps)
    t1 = time.perf_counter()
    s1, l1 = sess.stats(), sess.launch_counts()
    steps = s1["steps"] - s0["steps"]
    if steps <= 0:
        raise SystemExit("the search finished before the timed steps; lower --depth-steps")
    wall = t1 - t0
    launch = {"graph_replays": l1["graph_replays"] - l0["graph_replays"],
              "steps_per_replay": l1["steps_per_replay"],
              "direct_steps": l1["direct_steps"] - l0["direct_steps"]}
    # event window: the same number of steps right after, only the dominant
    # kernel bracketed by HIP events on the search stream (events recorded
    # inside a captured graph are not timed by this runtime, so these steps
    # launch one by one; a kernel's own duration does not depend on that)
    sess.set_profile(sum(1 << list(p1).index(n) for n in members))
    e0, k0 = sess.stats(), sess.kernel_times()
    te0 = time.perf_counter()
    sess.step(a.steps)
    te1 = time.perf_counter()
    e1, k1 = sess.stats(), sess.kernel_times()
    sess.set_profile(0)
    pairs = sum(s1[k] - s0[k] for k in ("frontier_pairs", "p_pairs", "group_pairs"))
    value = pairs / wall

    # the dominant kernel's launches over the event window
    ms_dom = sum(k1[n][0] - k0[n][0] for n in members)
    launches = k1[members[0]][1] - k0[members[0]][1]
    avg_s = ms_dom / 1e3 / max(launches, 1)
    ewin = e1["steps"] - e0["steps"]
    delta = {k: e1[k] - e0[k] for k in e1 if isinstance(e1[k], int)}
    nbytes = kernel_bytes(members[0], delta, d, ewin)
    nops = kernel_ops(dom, delta, d)
    bw = nbytes / max(launches, 1) / avg_s / 1e9          # GB/s
    ops = nops / max(launches, 1) / avg_s / 1e12          # TOP/s
    # the binding roof follows the kernel's arithmetic intensity (ops per byte)
    balance = ALU_PEAK_TOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = nops / nbytes if nbytes else (float("inf") if nops else 0.0)
    if intensity > balance:
        roof = {"bound": "alu", "achieved": ops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": ops / ALU_PEAK_TOPS, "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": bw, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": bw / HBM_PEAK_GBS, "traffic": None}
    roof["traffic"] = measured_traffic(dom, a.batch_width)
    roof["kernel"] = dom
    roof["avg_launch_us"] = avg_s * 1e6  # per step: both passes for the pair tiles
    roof["launches"] = launches
    roof["event_window"] = {"steps": ewin, "ms_per_step": 1e3 * (te1 - te0) / max(ewin, 1),
                            "launch": "one by one, dominant kernel bracketed by HIP events, "
                                      "right after the timed steps"}
    roof["bytes_per_launch"] = nbytes / max(launches, 1)
    roof["intensity_ops_per_byte"] = intensity
    if dom == PAIR_UNIT:
        roof["ops_model"] = ("2d int32 ops per (candidate, frontier entry or candidate) pair of "
                             "the large groups that the two pair passes decide, over their summed "
                             "duration per step; the second pass skips the rows of candidates "
                             "already rejected, so the vector units execute fewer (SQ instruction "
                             "counters of both passes in profiles/)")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "ship-routing grid 256x256, 8-connected, d=3 smooth-field costs, "
                               "corner to corner; one step = one batched label step",
                   "batch_width": a.batch_width, "label_steps_timed": steps,
                   "depth_steps": a.depth_steps, "search_finished": bool(done),
                   "steps_mode": "synchronous" if a.synchronous else "pipelined"},
        "timed_launches": launch,
        "roofline": roof,
        "kernel_us_per_step": {n: round(1e3 * v[0] / max(v[1], 1), 2)
                               for n, v in sorted(table.items(), key=lambda x: -x[1][0])},
        "kernel_table_steps": pre,
        "search_state": {"pops": s1["pops"], "labels": s1["inserted"], "front_so_far": s1["front"],
                         "pops_per_s": (s1["pops"] - s0["pops"]) / wall,
                         "labels_per_s": (s1["inserted"] - s0["inserted"]) / wall,
                         "tie_entries_per_step": (s1["tie_entries"] - s0["tie_entries"]) / steps,
                         "pairs_timed": pairs,
                         "pairs_timed_by_kind": {
                             k: s1[k] - s0[k] for k in ("frontier_pairs", "group_pairs",
                                                        "p_pairs", "pairs_onepass")},
                         "frontier_bytes_timed": s1["frontier_bytes"] - s0["frontier_bytes"]},
    }
    sess.close()
    if a.queries > 0:
        out["queries_per_s"] = batched_vs_plain(mos, gen, G, a)
    if a.time_to_front:
        out["time_to_exact_front"] = time_to_front(mos, gen)
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(g, s, t, a.cpu_seconds)
        if a.queries > 0:
            S, T = gen.ship_queries(256, 256, a.queries, seed=1000, dmin=a.qdist[0],
                                    dmax=a.qdist[1])
            out["cpu_baseline_all_cores"] = cpu_all_cores(g, S, T, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

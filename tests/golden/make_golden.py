"""Write expected Pareto fronts for the seeded workloads by calling the CPU oracle.

Every stored expected value under tests/golden/ that is not quoted from the
paper comes from this script, which calls only ``oracle`` (sequential NAMOA*)
and the seeded input generators ``gen``.

Usage:  python tests/golden/make_golden.py NAME [--time-limit S]
NAME is one of: c1_s<seed>, c1_all, ship<size>, c2, c3, c4_<first>_<count>, c4mid, route<r>,
      c2_prefix, c3_prefix, c4batch, c5_subset
  c1_all   the 32x32 grid query for seeds 0..31 (c1/s<seed>.txt.gz)
  c4mid    20 queries on the 256x256 ship grid with Manhattan distance in
           [60, 120] (query seed 99); the ones the oracle finishes within the
           time limit (default 10 s) are written to c4mid/q<i>.txt.gz
  route<r> the time-expanded route r (1..5) shaped like Table 2's route r, at
           that route's largest objective count in Table 2 (routes/r<r>.txt.gz)
  c2_prefix, c3_prefix  the full-size ship-grid and road-like queries: the
           oracle stopped after the time limit (default 600 s); the file holds
           its front so far below the bound it reports (an exact prefix)
  c4batch  the 512-query batch of the ship grid, each query time-boxed
           (default 20 s): complete fronts or exact prefixes
  c5_subset  200 random pairs on the 1M-node road-like graph, a third each at
           d = 3, 4, 5, time-boxed (default 20 s)
  trim:FILE  cut every entry of the stored set FILE (relative to this folder)
           to an exact prefix of at most --max-rows rows
"""
from __future__ import annotations

import argparse
import gzip
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = oracle.WEAK_P | oracle.LAZY_PRUNEOPEN


def write_front(path, header: dict, costs: np.ndarray):
    opener = gzip.open if path.endswith(".gz") else open
    with opener(path, "wt") as f:
        for k, v in header.items():
            f.write(f"# {k}: {v}\n")
        for row in costs:
            f.write(" ".join(str(int(x)) for x in row) + "\n")


def read_front(path):
    """Returns (header dict, int64 costs[size, d])."""
    opener = gzip.open if path.endswith(".gz") else open
    header, rows = {}, []
    with opener(path, "rt") as f:
        for line in f:
            if line.startswith("#"):
                k, _, v = line[1:].partition(":")
                header[k.strip()] = v.strip()
            elif line.strip():
                rows.append([int(x) for x in line.split()])
    d = int(header["d"])
    return header, np.array(rows, dtype=np.int64).reshape(-1, d)


def write_front_set(path, header: dict, entries: list):
    """Several queries' fronts in one gzip text file: a '#' header for the set,
    then per query an '@' line of key=value fields and its cost rows.  An
    entry with complete=0 holds the prefix of an early-stopped search and its
    bound (the F of the smallest label left in OPEN, space separated)."""
    with gzip.open(path, "wt") as f:
        for k, v in header.items():
            f.write(f"# {k}: {v}\n")
        for e, costs in entries:
            f.write("@ " + " ".join(f"{k}={v}" for k, v in e.items()) + "\n")
            for row in costs:
                f.write(" ".join(str(int(x)) for x in row) + "\n")


def read_front_set(path):
    """Returns (header dict, [(entry dict, int64 costs[size, d]), ...]); an
    entry's 'bound' field, when present, is an int64 array."""
    header, entries, cur, rows = {}, [], None, []

    def flush():
        if cur is not None:
            d = int(cur["d"])
            entries.append((cur, np.array(rows, dtype=np.int64).reshape(-1, d)))

    with gzip.open(path, "rt") as f:
        for line in f:
            if line.startswith("#"):
                k, _, v = line[1:].partition(":")
                header[k.strip()] = v.strip()
            elif line.startswith("@"):
                flush()
                cur, rows = {}, []
                for kv in line[1:].split():
                    k, _, v = kv.partition("=")
                    cur[k] = v
                if "bound" in cur:
                    cur["bound"] = np.array([int(x) for x in cur["bound"].split(",")], np.int64)
            elif line.strip():
                rows.append([int(x) for x in line.split()])
    flush()
    return header, entries


def truncate_entry(e: dict, rows, max_rows: int):
    """Keep at most max_rows rows of an entry (rows ascending): the dropped
    part is replaced by a bound, the first dropped row, below which the kept
    rows are still exactly the front (a prefix of a prefix is a prefix)."""
    if rows.shape[0] <= max_rows:
        return e, rows
    e = dict(e)
    e["complete"] = 0
    e["bound"] = ",".join(str(int(x)) for x in rows[max_rows])
    e["front"] = max_rows
    e["truncated_from"] = rows.shape[0]
    return e, rows[:max_rows]


def solve_set(g, S, T, D, time_limit, threads=8):
    """Oracle fronts of many queries on one graph, one query per thread (the
    oracle releases the interpreter while it searches).  A query the oracle
    does not finish within time_limit keeps its early-stopped prefix."""
    from concurrent.futures import ThreadPoolExecutor

    def one(q):
        r = oracle.solve(g, int(S[q]), int(T[q]), int(D[q]), flags=FLAGS, time_limit=time_limit,
                         want_paths=False)
        e = {"q": q, "start": int(S[q]), "goal": int(T[q]), "d": int(D[q]),
             "complete": int(r.status == "ok"), "pops": r.stats["pops"],
             "pairs": r.stats["frontier_pairs"] + r.stats["p_pairs"],
             "search_seconds": round(r.stats["search_seconds"], 3)}
        rows = r.costs
        if r.status != "ok":
            if r.open_min is None:
                raise SystemExit(f"query {q}: oracle {r.status}")
            bound, rows = oracle.prefix_bound(r)
            e["bound"] = ",".join(str(int(x)) for x in bound)
        e["front"] = len(rows)
        print(q, e["complete"], e["front"], e["search_seconds"], flush=True)
        return e, rows

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(S))))


def solve_one(name, g, s, t, d, time_limit):
    t0 = time.time()
    r = oracle.solve(g, s, t, d, flags=FLAGS, time_limit=time_limit)
    if r.status != "ok":
        raise SystemExit(f"{name}: oracle {r.status} after {time.time() - t0:.0f}s")
    header = {"workload": name, "graph": g.name, "graph_sha256_16": g.digest(),
              "start": s, "goal": t, "d": d, "oracle_flags": FLAGS,
              "front": r.stats["front"], "pops": r.stats["pops"],
              "pairs": r.stats["frontier_pairs"] + r.stats["p_pairs"],
              "search_seconds": round(r.stats["search_seconds"], 3)}
    return header, r.costs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--time-limit", type=float, default=0.0)
    ap.add_argument("--threads", type=int, default=8, help="queries solved at once (sets)")
    ap.add_argument("--max-rows", type=int, default=0,
                    help="sets: rows kept per query (0 = all); longer fronts and prefixes "
                         "are cut to an exact prefix of this many rows")
    a = ap.parse_args()
    name = a.name
    if name.startswith("c1_s"):
        seed = int(name[4:])
        g, s, t = gen.config1(seed)
        h, c = solve_one(name, g, s, t, 3, a.time_limit)
        write_front(os.path.join(HERE, f"{name}.txt"), h, c)
    elif name == "c1_all":
        os.makedirs(os.path.join(HERE, "c1"), exist_ok=True)
        for seed in range(32):
            g, s, t = gen.config1(seed)
            h, c = solve_one(f"c1_s{seed}", g, s, t, 3, a.time_limit)
            write_front(os.path.join(HERE, "c1", f"s{seed:02d}.txt.gz"), h, c)
            print(seed, h["front"], h["search_seconds"], flush=True)
    elif name == "c4mid":
        os.makedirs(os.path.join(HERE, "c4mid"), exist_ok=True)
        g = gen.ship_grid(256, 256, 3, 0)
        S, T = gen.ship_queries(256, 256, 20, seed=99, dmin=60, dmax=120)
        limit = a.time_limit or 10.0
        for q in range(20):
            r = oracle.solve(g, int(S[q]), int(T[q]), 3, flags=FLAGS, time_limit=limit)
            if r.status != "ok":
                print(q, r.status, flush=True)
                continue
            h = {"workload": f"c4mid_q{q}", "graph": g.name, "graph_sha256_16": g.digest(),
                 "start": int(S[q]), "goal": int(T[q]), "d": 3, "oracle_flags": FLAGS,
                 "front": r.stats["front"], "pops": r.stats["pops"],
                 "pairs": r.stats["frontier_pairs"] + r.stats["p_pairs"],
                 "search_seconds": round(r.stats["search_seconds"], 3)}
            write_front(os.path.join(HERE, "c4mid", f"q{q:02d}.txt.gz"), h, r.costs)
            print(q, h["front"], h["search_seconds"], flush=True)
    elif name.startswith("ship"):
        size = int(name[4:])
        g, s, t = gen.config2(0, size=size)
        h, c = solve_one(name, g, s, t, 3, a.time_limit)
        write_front(os.path.join(HERE, f"{name}.txt"), h, c)
    elif name == "c2":
        g, s, t = gen.config2(0)
        h, c = solve_one(name, g, s, t, 3, a.time_limit)
        write_front(os.path.join(HERE, "c2.txt.gz"), h, c)
    elif name == "c3":
        g, s, t = gen.config3(0)
        h, c = solve_one(name, g, s, t, 4, a.time_limit)
        write_front(os.path.join(HERE, "c3.txt.gz"), h, c)
    elif name.startswith("c4_"):
        first, count = (int(x) for x in name[3:].split("_"))
        g, S, T = gen.config4(0)
        for q in range(first, first + count):
            h, c = solve_one(f"c4_q{q}", g, int(S[q]), int(T[q]), 3, a.time_limit)
            write_front(os.path.join(HERE, "c4", f"q{q:03d}.txt"), h, c)
            print(q, h["front"], h["search_seconds"], flush=True)
    elif name in ("c2_prefix", "c3_prefix"):
        # the full-size single queries: the oracle's early-stopped prefix
        g, s, t = gen.config2(0) if name == "c2_prefix" else gen.config3(0)
        d = 3 if name == "c2_prefix" else 4
        limit = a.time_limit or 600.0
        res = solve_set(g, [s], [t], [d], limit, threads=1)
        hdr = {"workload": name, "graph": g.name, "graph_sha256_16": g.digest(), "d": d,
               "oracle_flags": FLAGS, "time_limit": limit}
        write_front_set(os.path.join(HERE, f"{name}.txt.gz"), hdr, res)
    elif name == "c4batch":
        # the 512-query batch as generated, every query time-boxed
        g, S, T = gen.config4(0)
        limit = a.time_limit or 20.0
        res = solve_set(g, S, T, [3] * len(S), limit, threads=a.threads)
        if a.max_rows:
            res = [truncate_entry(e, r, a.max_rows) for e, r in res]
        hdr = {"workload": name, "graph": g.name, "graph_sha256_16": g.digest(), "d": 3,
               "oracle_flags": FLAGS, "time_limit": limit, "queries": len(S)}
        write_front_set(os.path.join(HERE, "c4batch.txt.gz"), hdr, res)
    elif name == "c5_subset":
        # 200 uniformly random pairs on the 1M-node graph, d-stratified (each
        # of d = 3, 4, 5 takes a third), time-boxed
        g, rng, comp = gen.config5_graph(0)
        S, T, D = gen.c5_parity_queries(g, comp, 200, seed=0)
        limit = a.time_limit or 20.0
        res = solve_set(g, S, T, D, limit, threads=a.threads)
        if a.max_rows:
            res = [truncate_entry(e, r, a.max_rows) for e, r in res]
        hdr = {"workload": name, "graph": g.name, "graph_sha256_16": g.digest(), "d": 5,
               "oracle_flags": FLAGS, "time_limit": limit, "queries": len(S)}
        write_front_set(os.path.join(HERE, "c5_subset.txt.gz"), hdr, res)
    elif name.startswith("trim:"):
        # cut a stored set's entries to exact prefixes of at most --max-rows
        # rows (complete fronts and early-stopped prefixes alike)
        path = os.path.join(HERE, name[5:])
        hdr, entries = read_front_set(path)
        out = []
        for e, rows in entries:
            e = dict(e)
            if "bound" in e:
                e["bound"] = ",".join(str(int(x)) for x in e["bound"])
            out.append(truncate_entry(e, rows, a.max_rows))
        hdr["max_rows"] = a.max_rows
        write_front_set(path, hdr, out)
        print(name, sum(r.shape[0] for _, r in out), "rows kept")
    elif name.startswith("route"):
        r = int(name[5:])
        d = gen.ROUTE_MAX_OBJECTIVES[r]
        g, s, t = gen.tmplar_route(r, 12, 0)
        h, c = solve_one(f"route{r}_d{d}", g, s, t, d, a.time_limit)
        os.makedirs(os.path.join(HERE, "routes"), exist_ok=True)
        write_front(os.path.join(HERE, "routes", f"r{r}.txt.gz"), h, c)
        print(r, d, h["front"], h["pops"], h["search_seconds"], flush=True)
    else:
        raise SystemExit(f"unknown workload {name}")


if __name__ == "__main__":
    main()

"""Write expected Pareto fronts for the seeded workloads by calling the CPU oracle.

Every stored expected value under tests/golden/ that is not quoted from the
paper comes from this script, which calls only ``oracle`` (sequential NAMOA*)
and the seeded input generators ``gen``.

Usage:  python tests/golden/make_golden.py NAME [--time-limit S]
NAME is one of: c1_s<seed>, c1_all, ship<size>, c2, c3, c4_<first>_<count>, c4mid, route<r>
  c1_all   the 32x32 grid query for seeds 0..31 (c1/s<seed>.txt.gz)
  c4mid    20 queries on the 256x256 ship grid with Manhattan distance in
           [60, 120] (query seed 99); the ones the oracle finishes within the
           time limit (default 10 s) are written to c4mid/q<i>.txt.gz
  route<r> the time-expanded route r (1..5) shaped like Table 2's route r, at
           that route's largest objective count in Table 2 (routes/r<r>.txt.gz)
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


def solve_one(name, g, s, t, d, time_limit):
    t0 = time.time()
    r = oracle.solve(g, s, t, d, flags=FLAGS, time_limit=time_limit)
    if r.status != "ok":
        raise SystemExit(f"{name}: oracle {r.status} after {time.time() - t0:.0f}s")
    header = {"workload": name, "graph": g.name, "graph_sha256_16": g.digest(),
              "start": s, "goal": t, "d": d, "oracle_flags": FLAGS,
              "front": r.stats["front"], "pops": r.stats["pops"],
              "search_seconds": round(r.stats["search_seconds"], 3)}
    return header, r.costs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--time-limit", type=float, default=0.0)
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

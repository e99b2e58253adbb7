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

Prints one JSON line.  Also reports the roofline of the dominant kernel (kernel
durations from HIP events over the timed steps) and the CPU oracle's check
rate on a bounded sample of the same query.
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
    ap.add_argument("--warmup", type=int, default=300, help="untimed label steps before timing")
    ap.add_argument("--batch-width", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="length of the oracle sample for the CPU baseline (0 = skip)")
    return ap.parse_args()


def cpu_baseline(g, s, t, seconds):
    import oracle

    r = oracle.solve(g, s, t, 3, flags=oracle.WEAK_P | oracle.LAZY_PRUNEOPEN, time_limit=seconds)
    st = r.stats
    pairs = st["frontier_pairs"] + st["p_pairs"]
    secs = max(st["search_seconds"], 1e-9)
    return {"value": pairs / secs, "unit": "checks/s", "cores": 1, "kind": "oracle",
            "sample": f"first {secs:.1f} s of the sequential search of the same query "
                      f"({st['pops']} labels processed, {pairs} pair checks)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); queries shard "
              "across GPUs with no exchange, see the design notes", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    import gen
    import paper_2411_16667_amd as mos

    g, s, t = gen.config2(0)
    G = mos.Graph.from_gen(g)
    d = 3
    sess = mos.Session(G, s, t, batch_width=a.batch_width, profile_kernels=True,
                       steps_per_poll=16)
    if a.warmup:
        sess.step(a.warmup)
    s0, k0 = sess.stats(), sess.kernel_times()
    t0 = time.perf_counter()
    done = sess.step(a.steps)
    t1 = time.perf_counter()
    s1, k1 = sess.stats(), sess.kernel_times()
    steps = s1["steps"] - s0["steps"]
    if steps <= 0:
        raise SystemExit("the search finished before the timed steps; lower --warmup")
    wall = t1 - t0
    pairs = sum(s1[k] - s0[k] for k in ("frontier_pairs", "p_pairs", "group_pairs"))
    value = pairs / wall

    # per-kernel durations over the timed steps (HIP events on the search stream)
    kern = {n: (k1[n][0] - k0[n][0], k1[n][1] - k0[n][1]) for n in k1}
    dom = max(kern, key=lambda n: kern[n][0])
    ms_dom, launches = kern[dom]
    avg_s = ms_dom / 1e3 / max(launches, 1)
    fb = s1["frontier_bytes"] - s0["frontier_bytes"]
    fb1 = s1["frontier_bytes_onepass"] - s0["frontier_bytes_onepass"]
    if dom == "k_group_process":
        # algorithmic bytes: 4d per (candidate group, live frontier entry);
        # algorithmic ops: 2d int32 comparisons per candidate pair (<= both ways)
        nbytes = fb1
        nops = 2 * d * (s1["pairs_onepass"] - s0["pairs_onepass"])
    elif dom == "k_group_finish":
        nbytes, nops = fb - fb1, 0
    else:
        # goal-front pairs: d int32 comparisons each, operands staged in LDS
        nbytes, nops = 0, d * (s1["p_pairs"] - s0["p_pairs"])
    bw = nbytes / max(launches, 1) / avg_s / 1e9          # GB/s
    ops = nops / max(launches, 1) / avg_s / 1e12          # TOP/s
    # the binding roof follows the kernel's arithmetic intensity (ops per byte)
    balance = ALU_PEAK_TOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = nops / nbytes if nbytes else float("inf")
    if intensity > balance:
        roof = {"bound": "alu", "achieved": ops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": ops / ALU_PEAK_TOPS, "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": bw, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": bw / HBM_PEAK_GBS, "traffic": None}
    roof["intensity_ops_per_byte"] = intensity
    roof["hbm_gbs"] = bw
    roof["alu_tops"] = ops
    roof["kernel"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = launches

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
                   "search_finished": bool(done)},
        "roofline": roof,
        "kernels_ms": {n: round(v[0], 3) for n, v in sorted(kern.items(), key=lambda x: -x[1][0])},
        "search_state": {"pops": s1["pops"], "labels": s1["inserted"], "front_so_far": s1["front"],
                         "pairs_timed": pairs, "frontier_bytes_timed": fb},
    }
    sess.close()
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(g, s, t, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

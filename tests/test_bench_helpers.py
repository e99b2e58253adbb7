"""The bench's bookkeeping on the CPU: the kernel-source digest that keys the
committed HBM-traffic counters follows the code, not its comments, and the
committed summary is read back only for its own batch width."""
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _copy_sources(tmp):
    for f in bench.KERNEL_SOURCES:
        dst = os.path.join(tmp, f)
        os.makedirs(os.path.dirname(dst), exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), dst)


def test_digest_ignores_comments_not_code(tmp_path, monkeypatch):
    _copy_sources(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_source_digest()
    assert d0 == bench.kernel_source_digest()
    p = os.path.join(str(tmp_path), bench.KERNEL_SOURCES[0])
    with open(p, "a", encoding="utf-8") as f:
        f.write("\n// a note\n\n")
    assert bench.kernel_source_digest() == d0
    with open(p, "a", encoding="utf-8") as f:
        f.write("static int extra_symbol = 1;\n")
    assert bench.kernel_source_digest() != d0


def test_committed_traffic_summary_reads_back():
    text = open(bench.TRAFFIC_FILE, encoding="utf-8").read()
    meta = dict(line[2:].split(": ", 1) for line in text.splitlines()
                if line.startswith("- ") and ": " in line)
    bw = int(meta["batch width"])
    got = bench.measured_traffic("k_group_pairs", bw)
    if meta["kernel sources sha256/16"].split()[0] == bench.kernel_source_digest():
        assert got is not None and got > 0
    else:
        assert got is None  # counters of other kernel code are never reported
    assert bench.measured_traffic("k_group_pairs", bw + 1) is None
    assert bench.measured_traffic("no_such_kernel", bw) is None


def test_every_step_kernel_has_byte_accounting():
    """The benchmark's algorithmic-byte table names every kernel of the step
    (read from the library's own name table), so no kernel reports 0 bytes
    by omission."""
    import re

    src = open(os.path.join(ROOT, "paper_2411_16667_amd", "csrc", "step.hip")).read()
    table = src[src.index("kStepKernelNames[kStepKernels] = {"):]
    names = re.findall(r'"(k_\w+)"', table[:table.index("};")])
    csrc = os.path.join(ROOT, "paper_2411_16667_amd", "csrc")
    n = int(re.search(r"kStepKernels\s*=\s*(\d+) \+ NPASS",
                      open(os.path.join(csrc, "kernels.h")).read()).group(1))
    n += int(re.search(r"constexpr int NPASS = (\d+);",
                       open(os.path.join(csrc, "mos_core.h")).read()).group(1))
    assert len(names) == n == len(set(names))
    c = {k: 1 for k in ("pops", "killed", "candidates", "inserted", "frontier_bytes",
                        "frontier_bytes_onepass", "far_scanned", "near_scanned", "tie_entries",
                        "front_reads", "goal_pops", "pairs_onepass", "frontier_pairs",
                        "group_pairs", "p_pairs")}
    c["frontier_bytes"] = 2
    for k in names:
        assert bench.kernel_bytes(k, c, 3, 1) > 0 or k == "k_step_end", k
    assert bench.kernel_ops("k_group_pairs", c, 3) > 0
    assert bench.kernel_ops(bench.PAIR_UNIT, c, 3) > 0


def test_cpu_baseline_fields():
    """The CPU leg times the oracle on a bounded prefix and reports the
    contract's fields."""
    import gen

    g, s, t = gen.config1(0)
    r = bench.cpu_baseline(g, s, t, 0.5)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "checks/s"
    assert r["value"] > 0 and "labels processed" in r["sample"]

"""The oracle's pins catch plausible mistakes planted in the oracle.

Each case below plants one mistake (a transposed operand, a wrong index, a
dropped term, a prune taken out, a flag read the wrong way round) in a copy
of the oracle's source, builds it with g++ in a temporary folder and runs the
pin suite against that build in a child process.  The pins must fail.  A control run builds the unchanged source
the same way and must pass, so a failure is the mutant's and not the harness's.

Mutations that cannot change anything the search computes are left out on
purpose: with OPEN in lexicographic order and a consistent heuristic, a new
candidate never dominates a closed label (its parent had a smaller F), and
goal labels are popped in increasing cost order, so pruning the closed set
or the goal front on arrival is dead code there.  Some mutants change only
the work and not the front; the work pin (extractions counted by brute
force) is the one that catches those.
"""
import os
import resource
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "namoa.cpp")
# the rest of the oracle library, built unchanged beside each mutant
OTHER = [os.path.join(ROOT, "oracle", "necessary.cpp")]
PINS = os.path.join(HERE, "test_oracle_pins.py")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("cost planes read arc-major as plane-major",
     "gp[k] = gl[k] + g.cost[e * g.D + k];",
     "gp[k] = gl[k] + g.cost[k * g.m + e];"),
    ("operands transposed in the open-set dominance test",
     "for (int x : op) if (dominates(&lg[(i64)x * d], gp.data())) { domd = true; break; }",
     "for (int x : op) if (dominates(gp.data(), &lg[(i64)x * d])) { domd = true; break; }"),
    ("heuristic searched over forward arcs",
     "oracle_dijkstra(n, rptr.data(), rcol.data(), w.data(), goal, h + (i64)k * n);",
     "oracle_dijkstra(n, row_ptr, col, w.data(), goal, h + (i64)k * n);"),
    ("heuristic term dropped from F",
     "i64 F(int l, int k) const { return lg[(i64)l * d + k] + h[(i64)k * g.n + lv[l]]; }",
     "i64 F(int l, int k) const { return lg[(i64)l * d + k]; }"),
    ("heuristic of the parent node in F'",
     "Fp[k] = gp[k] + h[(i64)k * n + w];",
     "Fp[k] = gp[k] + h[(i64)k * n + v];"),
    ("dominated open label left in OPEN",
     "OPEN.erase(op[i]);\n",
     "\n"),
    ("goal-front test at pop with operands transposed",
     "if (p_rel(&lg[(i64)p * d], Fl.data())) { dead = true; break; }",
     "if (p_rel(Fl.data(), &lg[(i64)p * d])) { dead = true; break; }"),
    ("goal-front filter of a candidate tests g instead of F",
     "if (p_rel(&lg[(i64)p * d], Fp.data())) { ok = false; break; }",
     "if (p_rel(&lg[(i64)p * d], gp.data())) { ok = false; break; }"),
    ("strict and weak goal-front relations swapped",
     "return (flags & ORACLE_WEAK_P) ? weakly_dominates(p, x) : dominates(p, x);",
     "return (flags & ORACLE_WEAK_P) ? dominates(p, x) : weakly_dominates(p, x);"),
]

CHILD = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle
oracle.build = lambda force=False: {lib!r}
import pytest
sys.exit(pytest.main([{pins!r}, "-x", "-q", "-p", "no:cacheprovider",
                      "-k", "not config1"]))
"""


def _limit():
    # a mutant that blows up is stopped by the memory cap, not the machine
    resource.setrlimit(resource.RLIMIT_AS, (4 << 30, 4 << 30))


def _run_pins(tmp_path, source: str):
    cpp = tmp_path / "namoa.cpp"
    lib = tmp_path / "liboracle_mutant.so"
    cpp.write_text(source)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", str(lib),
                           str(cpp), *OTHER])
    code = CHILD.format(root=ROOT, tests=HERE, lib=str(lib), pins=PINS)
    return subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True,
                          text=True, timeout=120, preexec_fn=_limit)


def test_unchanged_oracle_passes_the_harness(tmp_path):
    r = _run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found once: " + name
    r = _run_pins(tmp_path, src.replace(old, new))
    # 1 = a pin failed (not a crash, a time-out or a harness error)
    assert r.returncode == 1, (name, r.returncode, r.stdout[-2000:])

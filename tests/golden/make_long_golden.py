"""Writes tests/golden/long_workload.txt: the oracle's results on the long-trace workload
(5 propositions, 4096 + 4096 traces of 64..512 positions, Bernoulli(0.3) letters, planted
formula of size 11, cost bound 13), seeds 0-3.

Calls only the CPU oracle (oracle/) and the seeded input generator (ltl_inputs/).  The
oracle runs in expansion mode (Sec. 4's backward recurrences, pinned against the
quantifier clauses in the CPU tests) with an OpenMP map over each level's candidates and
a sequential canonical-order merge, so results do not depend on the thread count.  A
full run takes about an hour on 6 cores and up to ~40 GB of host memory.

Usage: python tests/golden/make_long_golden.py [threads] [seeds...]
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O          # noqa: E402
from ltl_inputs import synth            # noqa: E402

OUT = os.path.join(HERE, "long_workload.txt")
HEADER = """\
# Oracle results on the long-trace workload (tests/golden/make_long_golden.py, which calls
# only oracle/ and ltl_inputs/): 5 props, 4096 + 4096 traces, lengths 64..512 (inclusive),
# Bernoulli(0.3) letters, labels from a planted formula of size 11, unit costs, cost bound 13.
# Sec. 3 enumeration with exact dedup (the exhaustive case of Sec. 5); canonical order
# F, U, G, X, And, Or, Not, splits ascending, pairs row-major.
#
# Format: seed :: status :: minimal cost :: levels done :: new languages per level 1.. ::
#         candidates per level 1.. :: canonical index of the first solution ::
#         solution as postfix nodes op,a,b separated by ';' (ops: 0 atom .. 7 U)
"""


def line(seed: int, threads: int) -> str:
    inst, cfg = synth.preset_instance("long", seed)
    r = O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND, threads=threads)
    d = r.levels_done
    sol = ";".join(f"{op},{a},{b}" for op, a, b in (r.solution or []))
    return " :: ".join([str(seed), str(r.status), str(r.cost), str(d),
                        ",".join(str(x) for x in r.level_new[1:d + 1]),
                        ",".join(str(x) for x in r.level_candidates[1:d + 1]),
                        str(r.first_index), sol or "-"])


def main(argv):
    threads = int(argv[1]) if len(argv) > 1 else 6
    seeds = [int(x) for x in argv[2:]] or [0, 1, 2, 3]
    have = {}
    if os.path.exists(OUT):
        for ln in open(OUT):
            if ln.strip() and not ln.startswith("#"):
                have[int(ln.split("::")[0])] = ln.rstrip("\n")
    for s in seeds:
        t0 = time.time()
        have[s] = line(s, threads)
        print(f"seed {s} done in {time.time() - t0:.0f} s: {have[s]}", flush=True)
        with open(OUT + ".tmp", "w") as fh:
            fh.write(HEADER)
            for k in sorted(have):
                fh.write(have[k] + "\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv)

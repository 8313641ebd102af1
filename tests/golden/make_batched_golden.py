"""Writes tests/golden/batched_mix.txt: the oracle's results on the first 64 jobs of the
batched workload (independent jobs of uneven size: 2..5 propositions, 16..2048 traces per
class, lengths 8..128, planted size 5..10, Bernoulli(0.5) letters, cost bound = planted
size + 2; ltl_inputs.synth.batched_jobs with master seed 0).

Calls only the CPU oracle (oracle/) and the seeded input generator (ltl_inputs/); expansion
mode, an OpenMP map over each level's candidates and a sequential canonical-order merge,
so results do not depend on the thread count.  About 5 minutes on 6 cores.

Usage: python tests/golden/make_batched_golden.py [threads] [njobs]
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

OUT = os.path.join(HERE, "batched_mix.txt")
HEADER = """\
# Oracle results on the first {n} jobs of the batched workload (tests/golden/make_batched_golden.py,
# which calls only oracle/ and ltl_inputs/): ltl_inputs.synth.batched_jobs(0), unit costs,
# every connective.  Sec. 3 enumeration with exact dedup; canonical order F, U, G, X, And,
# Or, Not, splits ascending, pairs row-major.
#
# Format: job :: cost bound :: status :: minimal cost :: levels done :: new languages per
#         level 1.. :: candidates per level 1.. :: canonical index of the first solution ::
#         solution as postfix nodes op,a,b separated by ';' (ops: 0 atom .. 7 U)
"""


def line(j: int, inst, bound: int, threads: int) -> str:
    r = O.learn(inst, bound, mode=O.MODE_EXPAND, threads=threads)
    d = r.levels_done
    sol = ";".join(f"{op},{a},{b}" for op, a, b in (r.solution or []))
    return " :: ".join([str(j), str(bound), str(r.status), str(r.cost), str(d),
                        ",".join(str(x) for x in r.level_new[1:d + 1]),
                        ",".join(str(x) for x in r.level_candidates[1:d + 1]),
                        str(r.first_index), sol or "-"])


def main(argv):
    threads = int(argv[1]) if len(argv) > 1 else 6
    n = int(argv[2]) if len(argv) > 2 else 64
    lines = []
    for j, (inst, bound) in enumerate(synth.batched_jobs(0, n)):
        t0 = time.time()
        lines.append(line(j, inst, bound, threads))
        print(f"job {j} done in {time.time() - t0:.1f} s", flush=True)
    with open(OUT + ".tmp", "w") as fh:
        fh.write(HEADER.format(n=n))
        for ln in lines:
            fh.write(ln + "\n")
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv)

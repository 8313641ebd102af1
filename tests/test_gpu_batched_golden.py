"""The batched workload on the batch executor against the oracle.

The first 64 jobs of the batched workload (ltl_inputs.synth.batched_jobs(0): 2..5
propositions, 16..2048 traces per class, lengths 8..128, planted size 5..10, bound = size
+ 2) run together on 4 lanes, device-resident as the bench runs them, with one shared
budget (regions sized per job, 64 GiB) and with equal slices (4 x 48 GiB).  Every job's status, minimal cost,
level counts, first canonical index and formula equal the oracle's stored results
(tests/golden/batched_mix.txt, written by tests/golden/make_batched_golden.py, which
calls only the oracle).
"""
from __future__ import annotations

import os

import pytest

from ltl_inputs import synth

pytestmark = pytest.mark.gpu


def _golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_mix.txt")
    out = {}
    for ln in open(path):
        if not ln.strip() or ln.startswith("#"):
            continue
        f = [x.strip() for x in ln.split("::")]
        j, bound, st, cost, done = (int(x) for x in f[:5])
        E = [int(x) for x in f[5].split(",")] if f[5] else []
        Cn = [int(x) for x in f[6].split(",")] if f[6] else []
        sol = None if f[8] == "-" else [tuple(int(v) for v in nd.split(",")) for nd in f[8].split(";")]
        out[j] = dict(bound=bound, status=st, cost=cost, done=done, E=E, C=Cn, first=int(f[7]), sol=sol)
    return out


GOLD = _golden()


@pytest.fixture(scope="module")
def ltl():
    from paper_2402_12373_amd import ltl as L
    return L


@pytest.mark.parametrize("mode", ["shared-budget", "slices"])
def test_batched_mix_matches_oracle(ltl, mode):
    jobs = synth.batched_jobs(0, len(GOLD))
    devs = [ltl.spec_to_device(inst) for inst, _ in jobs]
    bounds = [b for _, b in jobs]
    assert bounds == [GOLD[j]["bound"] for j in range(len(jobs))]
    flags = ltl.BATCH_SHARED_BUDGET if mode == "shared-budget" else 0
    print("batched mix", mode, len(jobs), "jobs", flush=True)
    # equal slices: each lane needs room for the largest job's solution level (job 60:
    # 1.7 M new languages of 19 KB at cost 9); a shared budget grows regions on demand
    import torch
    torch.cuda.empty_cache()
    ex = ltl.Batch(lanes=4, workspace_bytes=(64 << 30) if flags else (192 << 30), flags=flags)
    try:
        res, _, _ = ex.run(devs, bounds)
    finally:
        ex.close()
    for j, r in enumerate(res):
        want = GOLD[j]
        assert (r.status, r.levels_done) == (want["status"], want["done"]), j
        assert r.level_new[1:] == want["E"] and r.level_candidates[1:] == want["C"], j
        if want["status"] == 0:
            assert (r.cost, r.solution_index, r.solution) == (want["cost"], want["first"], want["sol"]), j

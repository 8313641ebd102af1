"""Parity at the benchmark's full sizes, in the configuration bench.py times.

* long workload, whole jobs to the minimal cost, seeds 0-3: status, minimal cost,
  every level's counts, the canonical index and formula of the first solution equal
  the oracle's stored results (tests/golden/long_workload.txt, written by
  tests/golden/make_long_golden.py, which calls only the oracle);
* scale workload (3 props, 1024+1024 traces, len 16..32, bound 11, 2^26 hash
  slots), the eight benchmark seeds: status, minimal cost, every level's counts
  and the first solution equal the oracle's (the oracle runs every level);
* long workload (5 props, 4096+4096 traces, len 64..512, multi-word 64-bit rows):
  levels 1..4 complete (counts, every entry's formula, sampled matrices), in the exact
  mode and with the relaxed check of Sec. 5 (full and 12-bit keyed sums, FKP keys);
* long workload, whole jobs with the relaxed check and full keys: the stored exact results.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import oracle as O
from ltl_inputs import synth

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def ltl():
    from paper_2402_12373_amd import ltl as L
    return L


@pytest.fixture(scope="module")
def big_ctx(ltl):
    # a long job's solution level (110 710 new languages of 327 KB at level 7) needs 36 GB
    c = ltl.Context(workspace_bytes=64 << 30, hash_slots_log2=26)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(8))
def test_scale_workload_full_parity(ltl, big_ctx, seed):
    inst, cfg = synth.preset_instance("scale", seed)
    print("scale seed", seed, flush=True)
    g = big_ctx.learn(ltl.spec_to_device(inst), cfg["bound"])
    o = O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND, threads=THREADS)
    assert (g.status, g.levels_done) == (o.status, o.levels_done)
    assert g.level_new == o.level_new[:o.levels_done + 1]
    assert g.level_candidates == o.level_candidates[:o.levels_done + 1]
    if o.status == O.ST_OK:
        assert g.cost == o.cost and g.solution_index == o.first_index and g.solution == o.solution
        assert g.cost <= cfg["size"]


@pytest.mark.parametrize("seed", [0, 1])
def test_long_workload_levels(ltl, big_ctx, seed):
    inst, cfg = synth.preset_instance("long", seed)
    print("long seed", seed, flush=True)
    run = O.Run(O.Spec.of(inst), 4, mode=O.MODE_EXPAND, threads=THREADS)
    ora = run.result()
    job = big_ctx.job(ltl.spec_to_device(inst), cfg["bound"])
    try:
        info = job.info()
        assert info.word_bits == 64
        for c in range(1, 5):
            st = job.eval_level(c)
            assert st.candidates == ora.level_candidates[c] and st.new_entries == ora.level_new[c], c
            n = ora.level_new[c]
            for e in range(n):
                assert job.formula(c, e) == run.entry_formula(c, e), (c, e)
            for e in sorted(set([0, n - 1] + list(range(0, n, max(1, n // 12))))):
                np.testing.assert_array_equal(job.dump_cm(c, e), run.entry_cm(c, e), err_msg=f"{c}/{e}")
    finally:
        job.close()


@pytest.mark.parametrize("kind,bits", [("hash", 0), ("hash", 12), ("fkp", 0)])
def test_long_workload_relaxed_levels(ltl, kind, bits):
    """The relaxed check (Sec. 5, keyed sums; FKP keys, Sec. 7) at the long workload's full
    size in the bench's relaxed configuration (2^26 slots, key seed 0; the row-split kernels
    with tiles spread over several workgroups), levels 1..4: the counts, every entry's
    formula and sampled stored matrices equal the oracle's relaxed run with the same keys.
    With keys cut to 12 bits, or FKP's first position of the first traces, false positives
    decide which languages are kept."""
    inst, cfg = synth.preset_instance("long", 0)
    print("long relaxed", kind, "key bits", bits, flush=True)
    okind = O.RUC_FKP if kind == "fkp" else O.RUC_HASH
    flags = ltl.CTX_RUC | (ltl.CTX_RUC_FKP if kind == "fkp" else 0)
    run = O.Run(O.Spec.of(inst), 4, mode=O.MODE_EXPAND, threads=THREADS, ruc=okind, ruc_seed=0, ruc_bits=bits)
    ora = run.result()
    c = ltl.Context(workspace_bytes=16 << 30, hash_slots_log2=26, flags=flags, ruc_seed=0, ruc_key_bits=bits)
    try:
        job = c.job(ltl.spec_to_device(inst), cfg["bound"])
        try:
            for lv in range(1, 5):
                st = job.eval_level(lv)
                assert st.candidates == ora.level_candidates[lv] and st.new_entries == ora.level_new[lv], lv
                n = ora.level_new[lv]
                for e in range(n):
                    assert job.formula(lv, e) == run.entry_formula(lv, e), (lv, e)
                for e in sorted(set([0, n - 1] + list(range(0, n, max(1, n // 8))))):
                    np.testing.assert_array_equal(job.dump_cm(lv, e), run.entry_cm(lv, e), err_msg=f"{lv}/{e}")
        finally:
            job.close()
    finally:
        c.close()
    if bits or kind == "fkp":
        assert sum(ora.level_new[1:5]) < sum(LONG_GOLDEN[0]["E"][:4])   # the exact counts


def _long_golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_workload.txt")
    out = {}
    if os.path.exists(path):
        for ln in open(path):
            if not ln.strip() or ln.startswith("#"):
                continue
            f = [x.strip() for x in ln.split("::")]
            seed, st, cost, done = (int(x) for x in f[:4])
            E = [int(x) for x in f[4].split(",")]
            Cn = [int(x) for x in f[5].split(",")]
            sol = None if f[7] == "-" else [tuple(int(v) for v in nd.split(",")) for nd in f[7].split(";")]
            out[seed] = dict(status=st, cost=cost, done=done, E=E, C=Cn, first=int(f[6]), sol=sol)
    return out


LONG_GOLDEN = _long_golden()


@pytest.mark.parametrize("seed", sorted(LONG_GOLDEN))
def test_long_workload_relaxed_whole_jobs(ltl, seed):
    """Whole long jobs with the relaxed check and full 126-bit keyed sums (levels 5..7 on the
    whole-row kernels): no two of these languages share a key, so the relaxed run keeps
    exactly the exact mode's languages and equals the oracle's stored exact results."""
    want = LONG_GOLDEN[seed]
    inst, cfg = synth.preset_instance("long", seed)
    print("long relaxed whole job, seed", seed, flush=True)
    c = ltl.Context(workspace_bytes=64 << 30, hash_slots_log2=26, flags=ltl.CTX_RUC, ruc_seed=0)
    try:
        g = c.learn(ltl.spec_to_device(inst), cfg["bound"])
    finally:
        c.close()
    assert (g.status, g.levels_done) == (want["status"], want["done"])
    assert g.level_new[1:] == want["E"] and g.level_candidates[1:] == want["C"]
    if want["status"] == 0:
        assert (g.cost, g.solution_index, g.solution) == (want["cost"], want["first"], want["sol"])


@pytest.mark.parametrize("seed", sorted(LONG_GOLDEN))
def test_long_workload_golden(ltl, big_ctx, seed):
    """Whole long-workload jobs (multi-word rows, U doubling across words, whole-row levels)
    against the oracle's results."""
    want = LONG_GOLDEN[seed]
    inst, cfg = synth.preset_instance("long", seed)
    print("long golden seed", seed, flush=True)
    g = big_ctx.learn(ltl.spec_to_device(inst), cfg["bound"])
    assert (g.status, g.levels_done) == (want["status"], want["done"])
    assert g.level_new[1:] == want["E"] and g.level_candidates[1:] == want["C"]
    if want["status"] == 0:
        assert (g.cost, g.solution_index, g.solution) == (want["cost"], want["first"], want["sol"])

"""GPU path vs the CPU oracle, element by element, through the C-ABI.

Bar: bit-exact.  Every compared quantity is integer: status, minimal cost,
per-level counts of new languages and of candidates, the canonical index and
formula of the first solution, and every stored characteristic matrix.
"""
from __future__ import annotations

import functools
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from ltl_inputs import synth
from ltl_text import load_canonical_cases, random_instance

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ltl():
    from paper_2402_12373_amd import ltl as L
    return L


@pytest.fixture(scope="module")
def ctx(ltl):
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=22)
    yield c
    c.close()


def _same(gpu, ora, where=""):
    assert gpu.status == ora.status, (where, gpu.status, ora.status)
    assert gpu.levels_done == ora.levels_done, (where, gpu.levels_done, ora.levels_done)
    for c in range(1, ora.levels_done + 1):
        assert gpu.level_new[c] == ora.level_new[c], (where, "E", c, gpu.level_new, ora.level_new)
        assert gpu.level_candidates[c] == ora.level_candidates[c], (where, "C", c)
    if ora.status == O.ST_OK:
        assert gpu.cost == ora.cost, where
        assert gpu.solution_index == ora.first_index, (where, gpu.solution_index, ora.first_index)
        assert gpu.solution == ora.solution, (where, gpu.solution, ora.solution)


@pytest.mark.parametrize("chunk", range(8))
def test_tiny_workload_parity(ctx, chunk):
    """Tiny planted workload (2 props, 16+16 traces, length 4..8, bound 7), 256 seeds."""
    for seed in range(chunk * 32, chunk * 32 + 32):
        inst, cfg = synth.preset_instance("tiny", seed)
        _say("tiny seed", seed)
        g = ctx.learn(inst, cfg["bound"])
        o = O.learn(inst, cfg["bound"])
        _same(g, o, f"tiny/{seed}")


@pytest.mark.parametrize("case", load_canonical_cases(), ids=lambda c: c["name"])
def test_canonical_order_cases(ctx, case):
    """Hand-derived first solutions of the Sec. 3 order (tests/golden/canonical_order.txt):
    the GPU returns the expected formula and canonical index."""
    _say("canonical order case", case["name"])
    g = ctx.learn(case["inst"], case["expect_cost"] + 1, cost=case["cost"], ops=case["op_mask"])
    assert (g.status, g.cost) == (0, case["expect_cost"]), case["name"]
    assert g.solution_index == case["expect_index"], (case["name"], g.solution_index)
    assert g.solution == case["expect_formula"], (case["name"], g.solution)


def _level_by_level(ltl, ctx, inst, bound, check_entries=True, max_entries_per_level=None, **oracle_kw):
    """Evaluates levels one at a time and compares every stored matrix and formula."""
    run = O.Run(O.Spec.of(inst), bound, mode=O.MODE_EXPAND, threads=8, **oracle_kw)
    ora = run.result()
    job = ctx.job(inst, bound)
    try:
        for c in range(1, ora.levels_done + 1):
            st = job.eval_level(c)
            assert st.new_entries == ora.level_new[c], (c, st.new_entries, ora.level_new[c])
            assert st.candidates == ora.level_candidates[c], c
            if not check_entries:
                continue
            n = ora.level_new[c]
            step = 1 if max_entries_per_level is None else max(1, n // max_entries_per_level)
            # a level with a solution, or at the bound, is not stored: formulas only
            assert st.stored == (st.first_solution == ltl.NO_SOLUTION and c < bound), c
            for e in range(0, n, step):
                assert job.formula(c, e) == run.entry_formula(c, e), (c, e)
                if st.stored:
                    np.testing.assert_array_equal(job.dump_cm(c, e), run.entry_cm(c, e),
                                                  err_msg=f"level {c} entry {e}")
            if not st.stored and n:
                with pytest.raises(ltl.LTLError):
                    job.dump_cm(c, 0)
        g = job.result()
    finally:
        job.close()
    _same(g, ora)
    return g, ora


def test_every_stored_matrix_tiny(ltl, ctx):
    for seed in (0, 2, 7):
        inst, cfg = synth.preset_instance("tiny", seed)
        _say("entries tiny", seed)
        _level_by_level(ltl, ctx, inst, 5)


LENGTH_SETS = [
    (1, 2, 3),
    (31, 32, 30),
    (33, 40, 64),
    (63, 64, 65),
    (127, 128, 129),
    (200, 511, 512),
    (1, 64, 129, 300),
]


@pytest.fixture(scope="module")
def ctx_whole(ltl):
    """Every level on the whole-row kernels (one wave per tile, one dispatch per class,
    separate write pass, member marking on levels that are not stored)."""
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=22, split_tiles=1)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_dbl(ltl):
    """U by the doubling of App. B at every level (multi-word rows default to the carry adder)."""
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=22, flags=ltl.CTX_U_DOUBLING)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_whole_dbl(ltl):
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=22, split_tiles=1, flags=ltl.CTX_U_DOUBLING)
    yield c
    c.close()


PATHS = ["row-split", "whole-row"]
PATHS_U = ["row-split", "whole-row", "row-split-doubling", "whole-row-doubling"]


def _pick(ctx, ctx_whole, path, ctx_dbl=None, ctx_whole_dbl=None):
    return {"row-split": ctx, "whole-row": ctx_whole, "row-split-doubling": ctx_dbl,
            "whole-row-doubling": ctx_whole_dbl}[path]


@pytest.mark.parametrize("path", PATHS_U)
@pytest.mark.parametrize("lengths", LENGTH_SETS, ids=lambda l: "len" + "-".join(map(str, l)))
def test_word_boundaries(ltl, ctx, ctx_whole, ctx_dbl, ctx_whole_dbl, lengths, path):
    """Traces straddling word boundaries (single and multi-word rows), all matrices to level 4,
    on the row-split kernels (what these small levels use by default) and forced onto the
    whole-row kernels, each with the U method chosen by row layout and with doubling forced."""
    rng = np.random.default_rng(sum(lengths))
    pos, neg = [], []
    for k in range(8):
        n = lengths[k % len(lengths)]
        tr = [int(x) for x in rng.integers(0, 4, size=n)]
        (pos if k % 2 == 0 else neg).append(tr)
    inst = synth.from_traces(pos, neg, 2)
    _say("boundaries", lengths, path)
    _level_by_level(ltl, _pick(ctx, ctx_whole, path, ctx_dbl, ctx_whole_dbl), inst, 4, max_entries_per_level=200)


@pytest.mark.parametrize("path", PATHS_U)
def test_until_chains_every_doubling_step(ltl, ctx, ctx_whole, ctx_dbl, ctx_whole_dbl, path):
    """p0 U p1 over runs of 64, 127-129, 255-257 and 511 positions (App. B doubling across
    64-position words; each step s = 64, 128, 256 is the first to set some bit, checked on
    the CPU in test_until_chains.py; the carry adder's prefix over up to 8 words of a
    trace): every stored matrix of levels 1-4 and every entry formula of level 5 equal the
    oracle's, with doubling forced and with the method chosen by row layout (the carry
    adder here)."""
    inst = synth.until_chain_instance(0)
    _say("until chains", path)
    g, _ = _level_by_level(ltl, _pick(ctx, ctx_whole, path, ctx_dbl, ctx_whole_dbl), inst, 5,
                           max_entries_per_level=400)
    assert g.level_new[1] == 2


@pytest.mark.parametrize("seed", [0, 5, 9])
def test_whole_row_tiny(ltl, ctx_whole, seed):
    """Tiny 32-bit levels forced onto the whole-row kernels: the learned result and every
    stored matrix equal the oracle's."""
    inst, cfg = synth.preset_instance("tiny", seed)
    _say("whole-row tiny", seed)
    _level_by_level(ltl, ctx_whole, inst, cfg["bound"])


@pytest.mark.parametrize("flags", ["lds-tiles", "lds-tiles-doubling"])
def test_whole_row_lds_tiles(ltl, flags):
    """The whole-row kernels with child operands of binary connectives staged in LDS for
    8 x 8 groups of pairs (LTL_CTX_LDS_TILES) on one-word and multi-word rows, both U
    methods: the oracle's results and every stored matrix."""
    fl = ltl.CTX_LDS_TILES | (ltl.CTX_U_DOUBLING if flags.endswith("doubling") else 0)
    c = ltl.Context(workspace_bytes=1 << 30, hash_slots_log2=20, split_tiles=1, flags=fl)
    try:
        for seed in (1, 4):
            inst, cfg = synth.preset_instance("tiny", seed)
            _say("lds tiles tiny", seed, flags)
            _level_by_level(ltl, c, inst, cfg["bound"])
        _say("lds tiles until chains", flags)
        _level_by_level(ltl, c, synth.until_chain_instance(0), 5, max_entries_per_level=200)
    finally:
        c.close()


def test_single_word_u64_rows(ltl):
    """Short traces in 64-bit words (one word per trace) match the 32-bit layout."""
    c64 = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=18, word_bits=64)
    try:
        for seed in range(8):
            inst, cfg = synth.preset_instance("tiny", seed)
            _same(c64.learn(inst, cfg["bound"]), O.learn(inst, cfg["bound"]), f"u64/{seed}")
    finally:
        c64.close()


@pytest.mark.parametrize("flags", ["carry", "doubling"])
@pytest.mark.parametrize("word_bits", [32, 64])
def test_u_carry_variant_matches(ltl, word_bits, flags):
    """Both U methods forced at every level, on 32-bit and 64-bit rows (and multi-word 64-bit
    rows of up to 200 positions): the oracle's results."""
    fl = ltl.CTX_U_CARRY if flags == "carry" else ltl.CTX_U_DOUBLING
    c = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=18, flags=fl, word_bits=word_bits)
    try:
        for seed in range(16):
            inst, cfg = synth.preset_instance("tiny", seed)
            _same(c.learn(inst, cfg["bound"]), O.learn(inst, cfg["bound"]), f"ucarry/{seed}")
        rng = np.random.default_rng(5)
        if word_bits == 64:
            inst = random_instance(rng, 2, 4, 4, 60, 200)
            _same(c.learn(inst, 4), O.learn(inst, 4, mode=O.MODE_EXPAND), "ucarry-long")
    finally:
        c.close()


@pytest.mark.parametrize("fp_bits", [1, 4, 12])
def test_forced_fingerprint_collisions(ltl, fp_bits):
    """Truncated fingerprints flood the exact compare and the fallback; results must not change."""
    c = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=18, fp_bits=fp_bits)
    try:
        total = 0
        for seed in range(6):
            inst, cfg = synth.preset_instance("tiny", seed)
            _say("fp_bits", fp_bits, "seed", seed)
            g = c.learn(inst, 6)
            _same(g, O.learn(inst, 6), f"fp{fp_bits}/{seed}")
            total += g.colliders
        assert total > 0
    finally:
        c.close()


@pytest.mark.parametrize("split_tiles", [0, 1], ids=PATHS)
def test_forced_collisions_multiword(ltl, split_tiles):
    """6-bit fingerprints on multi-word rows: the exact re-check (representatives'
    matrices, verification against them, the sequential fallback) on both kernel paths."""
    c = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=18, fp_bits=6, split_tiles=split_tiles)
    try:
        rng = np.random.default_rng(11)
        inst = random_instance(rng, 2, 3, 3, 70, 140)
        g = c.learn(inst, 4)
        _same(g, O.learn(inst, 4, mode=O.MODE_EXPAND), "fp6-long")
        assert g.colliders > 0
    finally:
        c.close()


def test_deterministic_reruns(ltl, ctx):
    inst, cfg = synth.preset_instance("tiny", 3)
    a = ctx.learn(inst, 7)
    b = ctx.learn(inst, 7)
    assert (a.status, a.cost, a.level_new, a.level_candidates, a.solution_index, a.solution) == \
           (b.status, b.cost, b.level_new, b.level_candidates, b.solution_index, b.solution)


def test_oom_entry_cap_matches_oracle(ltl):
    inst, cfg = synth.preset_instance("tiny", 0)
    for cap in (3, 10, 30):
        c = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=18, max_entries=cap)
        try:
            g = c.learn(inst, 7)
        finally:
            c.close()
        o = O.learn(inst, 7, max_entries=cap)
        assert g.status == o.status, (cap, g.status, o.status)
        assert g.levels_done == o.levels_done
        assert g.level_new == o.level_new[:o.levels_done + 1]


def test_invalid_specs(ltl, ctx):
    bad = [
        (synth.from_traces([[1, 2]], [[1, 2]], 2), ltl.LTL_E_INCONSISTENT),
        (synth.from_traces([[1, 2], []], [[3]], 2), ltl.LTL_E_INVAL),
        (synth.from_traces([[4]], [[1]], 2), ltl.LTL_E_INVAL),
        (synth.from_traces([[1] * 5000], [[0]], 1), ltl.LTL_E_TOO_LONG),
    ]
    for inst, st in bad:
        assert ctx.learn(inst, 3).status == st
    ok = synth.from_traces([[1, 0]], [[0, 1]], 1)
    r = ctx.learn(ok, 3)
    assert r.status == ltl.LTL_OK and r.cost == 1


def test_device_resident_spec(ltl, ctx):
    inst, cfg = synth.preset_instance("tiny", 9)
    dev = ltl.spec_to_device(inst)
    _same(ctx.learn(dev, 7), O.learn(inst, 7), "device-spec")


def test_level_calls_out_of_order(ltl, ctx):
    inst, cfg = synth.preset_instance("tiny", 1)
    job = ctx.job(inst, 7)
    try:
        with pytest.raises(ltl.LTLError):
            job.eval_level(2)
        job.eval_level(1)
    finally:
        job.close()


def test_table_reuse_across_jobs_after_oom(ltl):
    """A context hands its emptied hash table to the next job, also after an OOM stop."""
    c = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=16, max_entries=30)
    try:
        inst0, _ = synth.preset_instance("tiny", 0)
        g0 = c.learn(inst0, 7)
        assert g0.status == ltl.LTL_E_OOM
        for seed in (1, 2, 3, 4):
            inst, cfg = synth.preset_instance("tiny", seed)
            _same(c.learn(inst, 7), O.learn(inst, 7, max_entries=30), f"reuse/{seed}")
    finally:
        c.close()


@functools.lru_cache(maxsize=1)
def _scale3_oracle():
    inst, cfg = synth.preset_instance("scale", 3)
    return O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND, threads=8)


@pytest.mark.parametrize("split_tiles", [0, 1], ids=PATHS)
def test_arena_overflow_stops_and_context_recovers(ltl, split_tiles):
    """A level whose new languages do not fit the arena ends the job with LTL_E_OOM (the
    whole-row evaluation stops once the claims pass the arena): the completed levels equal
    the oracle's, and the same context then learns other jobs exactly."""
    inst, cfg = synth.preset_instance("scale", 3)       # level 8: 97 865 new languages of 8 KiB
    o = _scale3_oracle()
    c = ltl.Context(workspace_bytes=1 << 30, hash_slots_log2=22, split_tiles=split_tiles)
    try:
        g = c.learn(inst, cfg["bound"])
        _say("arena overflow", split_tiles, g.status, g.levels_done)
        assert g.status == ltl.LTL_E_OOM and 1 <= g.levels_done < o.levels_done
        assert g.level_new[1:] == o.level_new[1:g.levels_done + 1]
        assert g.level_candidates[1:] == o.level_candidates[1:g.levels_done + 1]
        for seed in (0, 5):
            inst2, cfg2 = synth.preset_instance("tiny", seed)
            _same(c.learn(inst2, cfg2["bound"]), O.learn(inst2, cfg2["bound"]), f"after overflow/{seed}")
    finally:
        c.close()


def test_batched_lanes_match_plain_runs(ltl):
    """ltl_learn_batch: every job's result equals its plain ltl_learn run (same slice size)."""
    jobs = [synth.preset_instance("tiny", s) for s in range(24)]
    insts = [j[0] for j in jobs]
    bounds = [j[1]["bound"] for j in jobs]
    lanes = 4
    ws = 1 << 30
    res, dur, done = ltl.learn_batch(insts, bounds, lanes=lanes, workspace_bytes=ws, hash_slots_log2=18)
    plain = ltl.Context(workspace_bytes=ws // lanes, hash_slots_log2=18)
    try:
        for inst, b, g in zip(insts, bounds, res):
            p = plain.learn(inst, b)
            assert (g.status, g.cost, g.level_new, g.level_candidates, g.solution_index, g.solution) == \
                   (p.status, p.cost, p.level_new, p.level_candidates, p.solution_index, p.solution)
            o = O.learn(inst, b)
            _same(g, o, "batched")
    finally:
        plain.close()
    assert all(d > 0 for d in dur) and max(done) >= max(dur)


def test_batch_executor_reuse(ltl):
    """ltl_batch_create/run: lanes kept across runs (tables reused); results equal plain runs."""
    jobs = [synth.preset_instance("tiny", s) for s in range(40, 60)]
    insts = [j[0] for j in jobs]
    bounds = [j[1]["bound"] for j in jobs]
    ex = ltl.Batch(lanes=3, workspace_bytes=768 << 20, hash_slots_log2=16, max_entries=3000)
    plain = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=16, max_entries=3000)
    try:
        first, _, _ = ex.run(insts[:12], bounds[:12])
        second, dur, done = ex.run(insts[8:], bounds[8:])
        bad, _, _ = ex.run(insts[:1], [0])              # a bad job fails alone; the run goes on
        assert bad[0].status == ltl.LTL_E_INVAL
        for inst, b, g in list(zip(insts[:12], bounds[:12], first)) + list(zip(insts[8:], bounds[8:], second)):
            p = plain.learn(inst, b)
            assert (g.status, g.cost, g.level_new, g.level_candidates, g.solution_index, g.solution) == \
                   (p.status, p.cost, p.level_new, p.level_candidates, p.solution_index, p.solution)
        assert len(dur) == 12 and all(d > 0 for d in dur)
    finally:
        ex.close()
        plain.close()


def _expected_alg_bytes(E, c, A, cm_bytes):
    """One matrix per candidate plus each child matrix once per tile of 4 x 4 (unit costs,
    every connective; F, G, X and NOT over one child level read the child once)."""
    ceil4 = lambda n: (n + 3) // 4
    if c == 1:
        return A, (A + A) * cm_bytes
    x = c - 1
    cands = reads = 0
    if E[x]:
        cands += 4 * E[x]
        reads += E[x]
    for a in range(1, x):                              # U: every ordered split
        na, nb = E[a], E[x - a]
        if na and nb:
            cands += na * nb
            reads += ceil4(nb) * na + ceil4(na) * nb
    for _ in range(2):                                 # AND, OR
        for a in range(1, x // 2 + 1):
            b = x - a
            na, nb = E[a], E[b]
            if a < b and na and nb:
                cands += na * nb
                reads += ceil4(nb) * na + ceil4(na) * nb
            elif a == b and na > 1:
                cands += na * (na - 1) // 2
                nt = ceil4(na)
                for it in range(nt):
                    rows = min(4, na - 4 * it)
                    reads += (nt - it) * rows + (it + 1) * rows
    return cands, (cands + reads) * cm_bytes


def test_level_algorithmic_bytes(ltl, ctx):
    """Per-level algorithmic bytes equal the model computed here from the level sizes."""
    inst, cfg = synth.preset_instance("tiny", 4)
    job = ctx.job(inst, 6)
    try:
        cm = int(job.info().cm_bytes)
        E = [0]
        for c in range(1, 7):
            st = job.eval_level(c)
            cands, want = _expected_alg_bytes(E, c, inst.num_props, cm)
            assert st.candidates == cands, c
            if not st.stored:                          # check-only: new entries are not written
                want -= st.new_entries * cm
            assert st.alg_bytes == want, (c, st.alg_bytes, want)
            E.append(st.new_entries)
            if st.first_solution != ltl.NO_SOLUTION:
                break
    finally:
        job.close()


@pytest.mark.parametrize("lo,hi", [(8, 32), (40, 120)], ids=["u32-4096-traces", "u64-multiword"])
def test_tiles_spread_over_workgroups(ltl, ctx, lo, hi):
    """Long rows and few tiles: a tile's row blocks span several workgroups (partial
    fingerprints added per candidate, claims by a probe pass, claimers written after)."""
    rng = np.random.default_rng(lo * 1000 + hi)
    inst = random_instance(rng, 2, 2048, 2048, lo, hi)
    _say("spread tiles", lo, hi)
    _level_by_level(ltl, ctx, inst, 4, max_entries_per_level=50)


def _mask(nnf, u_free):
    return ((O.ALL_OPS & ~(1 << 7)) if u_free else O.ALL_OPS) | (O.NNF if nnf else 0)


@pytest.mark.parametrize("nnf,u_free", [(True, True), (True, False), (False, True)],
                         ids=["nnf-ufree", "nnf", "ufree"])
def test_operator_sets_parity(ctx, nnf, u_free):
    """The operator sets of the experiments (Sec. 7): negation of atoms only, no U, or
    both; tiny planted workload, 32 seeds."""
    mask = _mask(nnf, u_free)
    for seed in range(32):
        inst, cfg = synth.preset_instance("tiny", seed)
        _say("operator set", hex(mask), "tiny seed", seed)
        g = ctx.learn(inst, cfg["bound"], ops=mask)
        o = O.learn(inst, cfg["bound"], op_mask=mask)
        _same(g, o, f"ops {mask:#x} tiny/{seed}")


@pytest.mark.parametrize("length,delta", [(3, 1), (3, 2), (4, 2)])
def test_hamming_parity(ltl, length, delta):
    """Hamming(B, l, delta) with the U-free NNF operator set (Sec. 7): one positive trace
    against every trace at bit distance delta.  Tiny matrices, minimal costs 10-15,
    levels of up to 1.4 M new languages."""
    c = ltl.Context(workspace_bytes=4 << 30, hash_slots_log2=24)
    try:
        for seed in range(2):
            inst = synth.hamming_instance(seed, length, delta)
            _say("hamming", length, delta, "seed", seed)
            g = c.learn(inst, 16, ops=O.U_FREE_NNF)
            o = O.learn(inst, 16, op_mask=O.U_FREE_NNF, mode=O.MODE_EXPAND, threads=16)
            _same(g, o, f"hamming/{length}/{delta}/{seed}")
            # short traces once gave distinct languages equal fingerprints (seed 1 of
            # length 4, distance 2: 37 pairs); the keyed premix leaves none here
            assert g.colliders == 0, (length, delta, seed, g.colliders)
    finally:
        c.close()


def test_batch_big_levels_take_turns(ltl):
    """LTL_BATCH_BIG_ALONE: lanes take turns for whole-row levels (scale jobs reach levels of
    10^5-10^6 candidates); every result equals the run without the flag and the plain run."""
    insts = [synth.preset_instance("scale", s)[0] for s in (3, 4, 1, 6)]
    dev = [ltl.spec_to_device(i) for i in insts]
    bound = synth.PRESETS["scale"]["bound"]
    key = lambda r: (r.status, r.cost, r.level_new, r.level_candidates, r.solution_index, r.solution)
    turns = ltl.Batch(lanes=3, workspace_bytes=48 << 30, hash_slots_log2=24, flags=ltl.BATCH_BIG_ALONE)
    free = ltl.Batch(lanes=3, workspace_bytes=48 << 30, hash_slots_log2=24)
    plain = ltl.Context(workspace_bytes=16 << 30, hash_slots_log2=24)
    try:
        a, _, _ = turns.run(dev, [bound] * len(dev))
        b, _, _ = free.run(dev, [bound] * len(dev))
        for i, (x, y) in enumerate(zip(a, b)):
            _say("big-alone job", i)
            assert key(x) == key(y), i
            assert key(x) == key(plain.learn(dev[i], bound)), i
        assert max(sum(1 for c in r.level_candidates if c >= 131072) for r in a) >= 1   # whole-row levels ran
    finally:
        turns.close()
        free.close()
        plain.close()


RUC_CASES = [("hash", 0), ("hash", 9), ("hash", 14), ("fkp", 0), ("fkp", 10)]
_RUC_ORACLE = {}      # oracle results per (case, key form, key bits), shared by the kernel paths


@pytest.mark.parametrize("split_tiles", [0, 1], ids=PATHS)
@pytest.mark.parametrize("kind,bits", RUC_CASES, ids=[f"{k}-{b or 126}bit" for k, b in RUC_CASES])
def test_relaxed_check_matches_oracle(ltl, kind, bits, split_tiles):
    """LTL_CTX_RUC (Sec. 5; FKP keys, Sec. 7) against the oracle's relaxed mode with the same
    126-bit keys: the same languages are cached (canonical-first candidate of each new key),
    so level counts, the first solution and its formula agree, on one-word and multi-word
    rows.  Keys cut to a few bits make false positives frequent, so the results depend on
    every key bit; slot hashes cut to 4 bits (fp_bits) make different keys share slots."""
    flags = ltl.CTX_RUC | (ltl.CTX_RUC_FKP if kind == "fkp" else 0)
    okind = O.RUC_FKP if kind == "fkp" else O.RUC_HASH
    rng = np.random.default_rng(5)
    cases = [(synth.preset_instance("tiny", s)[0], 7, None, f"tiny/{s}") for s in range(6)]
    cases.append((random_instance(rng, 2, 6, 6, 40, 150), 5, None, "u64 multi-word"))
    cases.append((random_instance(rng, 3, 5, 5, 60, 70), 5, None, "u64 one-word"))
    cases.append((random_instance(rng, 2, 4, 4, 3, 9), 7, None, "at most 126 bits"))
    # 3 traces of 33..40 positions, 115 bits: minimal cost 4
    cases.append((random_instance(np.random.default_rng(0), 1, 2, 1, 33, 40), 6, None, "at most 126 bits, 64-bit rows"))
    cases.append((synth.hamming_instance(0, 4, 2), 12, O.U_FREE_NNF, "hamming U-free NNF"))
    # long rows, few tiles: row-split tiles spread over several workgroups (partial sums)
    cases.append((synth.preset_instance("long", 0)[0], 3, None, "long rows"))
    for fp_bits in (0, 4):
        c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=20, flags=flags, ruc_seed=17,
                        ruc_key_bits=bits, fp_bits=fp_bits, split_tiles=split_tiles)
        try:
            for inst, bound, ops, name in cases:
                _say("ruc", kind, bits, fp_bits, name)
                key = (name, kind, bits)
                if key not in _RUC_ORACLE:
                    _RUC_ORACLE[key] = O.learn(inst, bound, op_mask=ops if ops is not None else O.ALL_OPS, ruc=okind,
                                               ruc_seed=17, ruc_bits=bits, mode=O.MODE_EXPAND, threads=8)
                o = _RUC_ORACLE[key]
                g = c.learn(inst, bound, ops=ops)
                _same(g, o, f"{kind}/{bits}/{fp_bits}/{name}")
                if bits == 0 and int(inst.offsets[-1]) <= 126:    # Sec. 5: exact up to 126 bits
                    _same(g, O.learn(inst, bound, op_mask=ops if ops is not None else O.ALL_OPS), name)
        finally:
            c.close()


def test_relaxed_check_row_split_small_rows(ltl):
    """The relaxed check on the row-split kernels forced at every level (the library keeps
    the whole-row kernels for short rows by default): the oracle's relaxed results."""
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=20, flags=ltl.CTX_RUC, ruc_seed=5, ruc_key_bits=9,
                    split_tiles=0xFFFFFFFF)
    try:
        for seed in range(6):
            inst, cfg = synth.preset_instance("tiny", seed)
            _say("ruc row-split tiny", seed)
            _same(c.learn(inst, cfg["bound"]), O.learn(inst, cfg["bound"], ruc=O.RUC_HASH, ruc_seed=5, ruc_bits=9),
                  f"ruc row-split/{seed}")
    finally:
        c.close()


@pytest.mark.parametrize("kind", ["hash", "fkp"])
def test_relaxed_check_stored_matrices(ltl, kind):
    """With truncated keys several languages share a key and the entry kept is the
    canonical-first one: every stored matrix and entry formula equals the oracle's."""
    flags = ltl.CTX_RUC | (ltl.CTX_RUC_FKP if kind == "fkp" else 0)
    okind = O.RUC_FKP if kind == "fkp" else O.RUC_HASH
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=20, flags=flags, ruc_seed=3, ruc_key_bits=11)
    try:
        rng = np.random.default_rng(9)
        for inst, bound, name in [(synth.preset_instance("tiny", 2)[0], 7, "tiny/2"),
                                  (random_instance(rng, 2, 6, 6, 40, 150), 5, "u64 multi-word")]:
            _say("ruc stored matrices", kind, name)
            _level_by_level(ltl, c, inst, bound, ruc=okind, ruc_seed=3, ruc_bits=11)
    finally:
        c.close()


def test_learn_complete(ltl, ctx, monkeypatch):
    """The learner of Sec. 3 (enumerate below the cost of overfitting, else return the
    overfitting formula).  Enumeration path: the oracle's result.  Fallback path: with the
    overfitting cost stubbed to 2 only the atom level is enumerated; no atom separates, so the
    result is the overfitting formula at that cost."""
    for seed in range(8):
        inst, cfg = synth.preset_instance("tiny", seed)
        r = ltl.learn_complete(ctx, inst)
        _, co = ltl.overfit(inst)
        o = O.learn(inst, min(co - 1, 63))
        _same(r, o, f"complete tiny/{seed}")
    inst = synth.from_traces([[1, 0]], [[1, 1], [0, 0], [1]], 1)
    assert O.learn(inst, 1).status == O.ST_NOT_FOUND
    nodes, _ = ltl.overfit(inst)
    monkeypatch.setattr(ltl, "overfit", lambda i, cost=None, ops=None: (nodes, 2))
    r = ltl.learn_complete(ctx, inst)
    assert (r.status, r.cost, r.solution, r.solution_index, r.levels_done) == (ltl.LTL_OK, 2, nodes, None, 1)


def _sound_by_oracle(inst, nodes):
    """The formula accepts every P trace and no N trace under the oracle's evaluator."""
    cm = O.eval_formula(O.Spec.of(inst), nodes, O.MODE_EXPAND)
    offs = inst.offsets.astype(np.int64)
    assert all(cm[offs[t]] for t in range(inst.num_pos))
    assert not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces))


def test_holds_matches_oracle(ltl, ctx):
    """ltl_holds (a given formula evaluated on the device) equals the oracle's position-0
    truth on single- and multi-word traces, for formulas of every connective."""
    rng = np.random.default_rng(42)
    for lo, hi in ((4, 8), (30, 70), (200, 512)):
        inst = random_instance(rng, 3, 12, 12, lo, hi)
        spec = O.Spec.of(inst)
        offs = inst.offsets.astype(np.int64)
        trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
        for size in (1, 3, 5, 7, 9):
            for k in range(6):
                nodes = synth.draw_formula(rng, size, 3)
                want = O.eval_formula(spec, nodes, O.MODE_QUANT)[offs[:-1]].astype(bool)
                got = ltl.holds(ctx, trs, nodes, 3)
                assert (got == want).all(), (lo, hi, nodes)
    with pytest.raises(ltl.LTLError):
        ltl.holds(ctx, [[1, 0]], [(ltl.ATOM, 5, 0)], 3)             # a missing proposition
    with pytest.raises(ltl.LTLError):
        ltl.holds(ctx, [[1, 0]], [(ltl.NOT, 0, 0)], 3)              # a child that is not earlier


@pytest.mark.parametrize("cap", [0, 40], ids=["no-cap", "entry-cap-40"])
def test_det_split_parity(ltl, cap):
    """Deterministic splitting (Sec. 6) over the GPU learner equals the same splitting over
    the oracle, formula for formula, for several windows; with an entry cap of 40 the large
    windows run out of memory and are halved on both sides alike."""
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=20, max_entries=cap)
    try:
        for seed in range(6):
            inst, cfg = synth.preset_instance("tiny", seed)
            offs = inst.offsets.astype(np.int64)
            trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
            P, N = trs[:inst.num_pos], trs[inst.num_pos:]
            for win in (3, 8, 32):
                _say("det_split seed", seed, "win", win, "cap", cap)
                g = ltl.det_split(c, P, N, inst.num_props, win)
                o = O.det_split(P, N, inst.num_props, win, max_entries=cap)
                assert g[0] == o[0] and g[1] == o[1], (seed, win, g, o)
                if g[0] == ltl.LTL_OK:
                    _sound_by_oracle(inst, g[1])
    finally:
        c.close()


@pytest.mark.parametrize("cap", [0, 40], ids=["no-cap", "entry-cap-40"])
def test_rand_split_parity(ltl, cap):
    """Random splitting (Sec. 6) in the library equals the oracle's driver formula for
    formula: both draw the random subsets from their own SplitMix64 streams (the same
    published generator); with an entry cap of 40 windows are halved on both sides alike."""
    c = ltl.Context(workspace_bytes=2 << 30, hash_slots_log2=20, max_entries=cap)
    try:
        for seed in range(6):
            inst, cfg = synth.preset_instance("tiny", seed)
            offs = inst.offsets.astype(np.int64)
            trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
            P, N = trs[:inst.num_pos], trs[inst.num_pos:]
            for win, rs in ((4, 0), (8, 1), (32, 2)):
                _say("rand_split seed", seed, "win", win, "cap", cap)
                g = ltl.rand_split(c, P, N, inst.num_props, win, seed=rs)
                o = O.rand_split(P, N, inst.num_props, win, seed=rs, max_entries=cap)
                assert g[0] == o[0] and g[1] == o[1], (seed, win, g, o)
                if g[0] == ltl.LTL_OK:
                    _sound_by_oracle(inst, g[1])
    finally:
        c.close()


def test_batch_serve_arrivals(ltl):
    """ltl_batch_serve: jobs start no earlier than they arrive, and every result equals the
    job's plain run, alone and in the mix."""
    jobs = [synth.preset_instance("tiny", s) for s in range(80, 104)]
    insts = [j[0] for j in jobs]
    bounds = [j[1]["bound"] for j in jobs]
    arrival = synth.poisson_arrivals(1, len(insts), 400.0)      # about 60 ms in all
    ex = ltl.Batch(lanes=3, workspace_bytes=768 << 20, hash_slots_log2=16)
    plain = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=16)
    key = lambda r: (r.status, r.cost, r.level_new, r.level_candidates, r.solution_index, r.solution)
    try:
        res, dur, done = ex.serve(insts, bounds, arrival)
        for i, (inst, b, g) in enumerate(zip(insts, bounds, res)):
            assert key(g) == key(plain.learn(inst, b)), i
            assert done[i] >= arrival[i] + dur[i] - 1e-3, (i, done[i], arrival[i], dur[i])
        with pytest.raises(ltl.LTLError):
            ex.serve(insts[:2], bounds[:2], [5.0, 1.0])                 # decreasing arrivals
    finally:
        ex.close()
        plain.close()


def test_autotune(ltl, ctx):
    """ltl_autotune times each tile shape / level schedule on a job and picks the fastest;
    every configuration gives the job's result (checked by the library), the context's own
    options are unchanged afterwards."""
    for inst, bound in ((synth.preset_instance("tiny", 3)[0], 7), (synth.until_chain_instance(0), 5)):
        best, rows = ctx.autotune(inst, bound)
        _say("autotune", inst.name, best, rows)
        assert len(rows) == 5 and all(ms > 0 for _, _, ms in rows)
        assert best in [(f, t) for f, t, _ in rows]
        assert ctx.opts.split_tiles == 0 and ctx.opts.flags == 0
        _same(ctx.learn(inst, bound), O.learn(inst, bound, mode=O.MODE_EXPAND), "after autotune")


def test_batch_shared_budget_admission(ltl):
    """LTL_BATCH_SHARED_BUDGET serving: jobs get regions of one 1 GiB budget sized by their
    estimated footprint (at least budget / 12 here); the regions in use never exceed the
    budget; a job that outgrows its region runs again in a larger one (the Hamming job of
    bound 12 needs a few hundred MB); every result equals the job's plain run alone on a
    context with the whole budget."""
    budget = 1 << 30
    specs = [synth.preset_instance("tiny", s) for s in range(12)]
    insts = [i for i, _ in specs] + [synth.hamming_instance(0, 4, 2), synth.until_chain_instance(0),
                                     synth.preset_instance("scale", 0)[0]]
    bounds = [c["bound"] for _, c in specs] + [12, 5, 11]
    arrival = synth.poisson_arrivals(3, len(insts), 200.0)
    ex = ltl.Batch(lanes=3, workspace_bytes=budget, flags=ltl.BATCH_SHARED_BUDGET)
    key = lambda r: (r.status, r.cost, r.levels_done, r.level_new, r.level_candidates, r.solution_index, r.solution)
    try:
        res, dur, done = ex.serve(insts, bounds, arrival)
        st = ex.stats()
        _say("shared budget: peak", st.peak_bytes, "reruns", st.reruns, "in flight", st.max_in_flight)
        assert 0 < st.budget_bytes <= budget and 0 < st.peak_bytes <= st.budget_bytes
        assert st.reruns >= 1 and st.admissions == len(insts) + st.reruns
        assert st.max_in_flight >= 2
        for i in range(len(insts)):
            assert done[i] >= arrival[i], i
    finally:
        ex.close()
    plain = ltl.Context(workspace_bytes=budget)
    try:
        for i, (inst, b) in enumerate(zip(insts, bounds)):
            assert key(res[i]) == key(plain.learn(inst, b)), i
    finally:
        plain.close()


@pytest.mark.gpu
def test_hamming_by_splitting(ltl):
    """Hamming specifications that the plain learner cannot finish, solved by deterministic
    and random splitting (Sec. 6) with the U-free operator set (negation anywhere: the
    overfitting formula of the leaves negates X): formula for formula the oracle's, and
    sound under the oracle's own evaluator."""
    mask = 0xFF & ~(1 << ltl.U)
    # room enough that no leaf runs out of memory (the oracle has no cap here)
    c = ltl.Context(workspace_bytes=64 << 30, hash_slots_log2=26)
    try:
        for length in (5, 6):
            inst = synth.hamming_instance(0, length, 2)
            offs = inst.offsets.astype(np.int64)
            trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
            P, N = trs[:1], trs[1:]
            for kind in ("det", "rand"):
                _say("hamming split", kind, "length", length)
                if kind == "det":
                    g = ltl.det_split(c, P, N, 2, 16, ops=mask)
                    o = O.det_split(P, N, 2, 16, op_mask=mask)
                else:
                    g = ltl.rand_split(c, P, N, 2, 16, seed=0, ops=mask)
                    o = O.rand_split(P, N, 2, 16, seed=0, op_mask=mask)
                assert g[0] == ltl.LTL_OK and g[0] == o[0] and g[1] == o[1], (kind, length, g, o)
                spec = O.Spec.of(synth.from_traces(P, N, 2))
                assert O.holds(spec, 0, 0, g[1])
                assert not any(O.holds(spec, t, 0, g[1]) for t in range(1, len(N) + 1))
    finally:
        c.close()

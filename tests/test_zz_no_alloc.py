"""ltl_learn_noalloc (learning on the library's fixed device scratch array, for callers
that cannot allocate) against ltl_learn on a caller workspace, through the C-ABI:
identical results on calls in a row, each call smaller than the one before, and a clear
error for a specification that does not fit the array."""
from __future__ import annotations

import numpy as np
import pytest

from ltl_inputs import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltl():
    from paper_2402_12373_amd import ltl as L
    return L


def _key(r):
    return (r.status, r.cost, r.levels_done, r.level_new, r.level_candidates, r.solution_index, r.solution)


def test_noalloc_matches_workspace_entry_point(ltl):
    ctx = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=ltl.NOALLOC_SLOTS_LOG2)
    try:
        tiny, cfg = synth.preset_instance("tiny", 5)
        offs = tiny.offsets.astype(np.int64)
        trs = [list(map(int, tiny.letters[offs[t]:offs[t + 1]])) for t in range(tiny.num_traces)]
        small = synth.from_traces(trs[:6], trs[tiny.num_pos:tiny.num_pos + 6], tiny.num_props)
        calls = [(synth.until_chain_instance(0), 5),        # multi-word 64-bit rows
                 (tiny, cfg["bound"]),                        # 32-bit rows, smaller
                 (small, cfg["bound"])]                       # smaller again
        for k, (inst, bound) in enumerate(calls):
            print("noalloc call", k, inst.name, inst.num_traces, "traces", flush=True)
            a = ltl.learn_noalloc(inst, bound)
            b = ctx.learn(inst, bound)
            assert a.status in (ltl.LTL_OK, ltl.LTL_NOT_FOUND), (k, a.status)
            assert _key(a) == _key(b), k
    finally:
        ctx.close()


def test_noalloc_rejects_what_does_not_fit(ltl):
    rng = np.random.default_rng(3)
    n, length = 5000, 4096                 # 82 MB of letters alone: more than the array
    print("noalloc oversize", n, "x", length, flush=True)
    letters = rng.integers(0, 4, size=n * length).astype(np.uint32)
    inst = synth.Instance(2, letters, np.arange(0, n * length + 1, length, dtype=np.uint64), n // 2, n - n // 2)
    r = ltl.learn_noalloc(inst, 3)
    assert r.status == ltl.LTL_E_OOM
    # the array is usable again afterwards
    tiny, cfg = synth.preset_instance("tiny", 2)
    ctx = ltl.Context(workspace_bytes=256 << 20, hash_slots_log2=ltl.NOALLOC_SLOTS_LOG2)
    try:
        assert _key(ltl.learn_noalloc(tiny, cfg["bound"])) == _key(ctx.learn(tiny, cfg["bound"]))
    finally:
        ctx.close()

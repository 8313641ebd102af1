"""The stored long-workload results (tests/golden/long_workload.txt) checked on the CPU:
each stored solution separates its specification under the oracle's evaluator and has the
stored minimal cost (unit costs: its node count), and the first levels' counts equal a
fresh oracle run."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from ltl_inputs import synth
from test_gpu_full_size import LONG_GOLDEN


@pytest.mark.parametrize("seed", sorted(LONG_GOLDEN))
def test_long_golden_is_consistent(seed):
    want = LONG_GOLDEN[seed]
    inst, cfg = synth.preset_instance("long", seed)
    assert want["status"] == O.ST_OK and want["done"] == want["cost"] <= cfg["size"]
    assert len(want["E"]) == len(want["C"]) == want["done"]
    sol = want["sol"]
    assert len(sol) == want["cost"]
    cm = O.eval_formula(O.Spec.of(inst), sol, O.MODE_EXPAND)
    offs = inst.offsets.astype(np.int64)
    assert cm[offs[:inst.num_pos]].all() and not cm[offs[inst.num_pos:-1]].any()
    upto = min(3, want["done"])
    r = O.learn(inst, upto, mode=O.MODE_EXPAND, threads=4)
    assert r.level_new[1:upto + 1] == want["E"][:upto]
    assert r.level_candidates[1:upto + 1] == want["C"][:upto]

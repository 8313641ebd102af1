"""The until-chain specification exercises every doubling step of App. B, checked on
the CPU through the oracle (no GPU): p0 U p1 is a cost-3 language of the specification
whose true positions need chains of 64, 127-129, 255-257 and 511 positions.

App. B's doubling sets a U bit whose until-chain (positions from i to the first psi)
has length d only at the step s = 2^floor(log2 d); with ceil(log2 512) = 9 steps the
last one (s = 256) is the only one that covers chains of 256..511 positions, so a
doubling with one step fewer, or with a wrong shift across 64-position words at s = 64,
128 or 256, gives a different matrix for this language.  The GPU tests compare every
stored matrix of this specification with the oracle's.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from ltl_inputs import synth

ATOM, U = 0, 7
P0_U_P1 = [(ATOM, 0, 0), (ATOM, 1, 0), (U, 0, 1)]


def _chain_lengths(inst, spec):
    """Until-chain length of every true position of p0 U p1 (from the oracle's
    matrices): distance to the first p1 at or after the position."""
    p0 = O.eval_formula(spec, [(ATOM, 0, 0)])
    p1 = O.eval_formula(spec, [(ATOM, 1, 0)])
    u = O.eval_formula(spec, P0_U_P1)
    out = []
    for t in range(inst.num_traces):
        a, b = int(inst.offsets[t]), int(inst.offsets[t + 1])
        for i in range(a, b):
            if not u[i]:
                continue
            j = i
            while not p1[j]:
                assert p0[j] and j + 1 < b, "a true U position has an unbroken p0 run ending in p1"
                j += 1
            out.append(j - i)
    return out


def test_until_chain_spec_needs_every_doubling_step():
    inst = synth.until_chain_instance(0)
    spec = O.Spec.of(inst)
    ks = int(np.ceil(np.log2(inst.max_len)))
    assert ks == 9
    d = set(_chain_lengths(inst, spec))
    for want in synth.UNTIL_CHAINS:
        assert want in d, want
    # every step s = 1, 2, ..., 256 is the first to set some bit
    for i in range(ks):
        s = 1 << i
        assert any(s <= x < 2 * s for x in d), s
    # chains of 256 or more: a doubling of ks - 1 steps misses them
    assert max(d) >= 1 << (ks - 1)


def test_until_chain_language_is_a_cost_3_entry():
    inst = synth.until_chain_instance(0)
    spec = O.Spec.of(inst)
    run = O.Run(spec, 3, mode=O.MODE_EXPAND)
    res = run.result()
    assert res.levels_done == 3 and res.level_new[1] == 2
    u = O.eval_formula(spec, P0_U_P1)
    assert any(np.array_equal(run.entry_cm(3, e), u) for e in range(res.level_new[3]))

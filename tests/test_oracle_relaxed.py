"""Pins of the oracle's relaxed uniqueness check (Sec. 5; FKP of Sec. 7).

The relaxed check caches a candidate iff its 126-bit key is new.  The key is the
matrix itself when the matrix has at most 126 bits (the check is then exact, as
Sec. 5 states), else the first-k-percent projection (FKP, Sec. 7) or a keyed hash.
What is pinned here, against facts other than the oracle's own code:
  * FKP's k for the paper's worked size (64 traces of 63 positions: k = 3, Sec. 7);
  * a hand-packed FKP key (two traces of 100 positions: 63 + 63 bits);
  * exactness when the matrix has at most 126 bits (both key forms give the exact
    learner's results, level by level);
  * the hash form reads every position: flipping any one bit changes the key;
  * truncated keys are the full key's leading bits, and a run never caches more
    languages than there are keys of that width;
  * soundness: a relaxed run's formula separates (textbook semantics) and costs at
    least the exact minimum; entries never share a key.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from ltl_inputs import synth
from ltl_text import random_instance


def _distinct_traces(rng, n, length, num_props=1):
    seen, out = set(), []
    while len(out) < n:
        t = tuple(int(x) for x in rng.integers(0, 1 << num_props, size=length))
        if t not in seen:
            seen.add(t)
            out.append(list(t))
    return out


def test_fkp_k_of_the_paper_example():
    """Sec. 7: for a CM of 64 traces of 63 positions FKP keeps k = 3 percent, 2 positions
    a trace (128 bits, the nearest total to 126)."""
    rng = np.random.default_rng(7)
    tr = _distinct_traces(rng, 64, 63)
    spec = O.Spec.of(synth.from_traces(tr[:32], tr[32:], 1))
    k, m = O.fkp_prefixes(spec)
    assert k == 3 and m == [2] * 64


def test_fkp_whole_matrix_when_it_fits():
    spec = O.Spec.of(synth.from_traces([[0, 1, 0]], [[1, 1]], 1))
    assert O.fkp_prefixes(spec) == (0, [3, 2])


def test_fkp_key_packed_by_hand():
    """Two traces of 100 positions: k = 63 keeps 63 + 63 positions, 126 bits exactly.
    Trace 0 true at 0..62, trace 1 true at 0 only: the key string is 64 ones, then 62 zeros."""
    rng = np.random.default_rng(3)
    tr = _distinct_traces(rng, 2, 100)
    spec = O.Spec.of(synth.from_traces([tr[0]], [tr[1]], 1))
    assert O.fkp_prefixes(spec) == (63, [63, 63])
    cm = np.zeros(200, dtype=np.uint8)
    cm[0:63] = 1
    cm[100] = 1
    want = ((1 << 64) - 1) << 62
    assert O.ruc_key(spec, cm, O.RUC_FKP) == want
    cm2 = cm.copy()
    cm2[63:100] = 1          # beyond trace 0's prefix: same key
    cm2[163:200] = 1         # beyond trace 1's prefix
    assert O.ruc_key(spec, cm2, O.RUC_FKP) == want
    cm3 = cm.copy()
    cm3[162] = 1             # trace 1, position 62: the key's last bit
    assert O.ruc_key(spec, cm3, O.RUC_FKP) == want | 1


def test_small_matrix_is_its_own_key():
    """At most 126 bits: both forms give the matrix, trace by trace, as the key."""
    spec = O.Spec.of(synth.from_traces([[1, 0, 1, 1]], [[0, 0, 1]], 1))
    cm = np.array([1, 0, 1, 1, 0, 1, 1], dtype=np.uint8)
    want = int("1011011", 2) << (126 - 7)
    assert O.ruc_key(spec, cm, O.RUC_FKP) == want
    assert O.ruc_key(spec, cm, O.RUC_HASH, seed=99) == want


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("ruc", [O.RUC_HASH, O.RUC_FKP])
def test_precise_when_matrix_fits_126_bits(seed, ruc):
    """Sec. 5: with at most 126 bits per matrix the relaxed check is exact."""
    rng = np.random.default_rng(100 + seed)
    inst = random_instance(rng, 2, 4, 4, 3, 9)
    assert int(inst.offsets[-1]) <= 126
    ex = O.learn(inst, 7)
    rx = O.learn(inst, 7, ruc=ruc, ruc_seed=seed)
    assert (rx.status, rx.cost, rx.levels_done, rx.first_index, rx.solution) == \
           (ex.status, ex.cost, ex.levels_done, ex.first_index, ex.solution)
    assert rx.level_new == ex.level_new and rx.level_candidates == ex.level_candidates


def test_hash_key_reads_every_position():
    """Each 32-position chunk enters its own odd-keyed product, so a change of any one
    position changes the key (a dropped chunk, trace or tail would not)."""
    rng = np.random.default_rng(11)
    inst = random_instance(rng, 2, 3, 3, 20, 70)
    spec = O.Spec.of(inst)
    tb = spec.tb
    assert tb > 126
    cm = (rng.random(tb) < 0.5).astype(np.uint8)
    base = O.ruc_key(spec, cm, O.RUC_HASH, seed=5)
    keys = {base}
    for q in range(tb):
        c2 = cm.copy()
        c2[q] ^= 1
        k = O.ruc_key(spec, c2, O.RUC_HASH, seed=5)
        assert k != base, q
        keys.add(k)
    assert len(keys) == tb + 1
    # the seed selects the keyed sums
    assert O.ruc_key(spec, cm, O.RUC_HASH, seed=6) != base


@pytest.mark.parametrize("ruc", [O.RUC_HASH, O.RUC_FKP])
def test_truncated_key_is_the_leading_bits(ruc):
    rng = np.random.default_rng(12)
    inst = random_instance(rng, 2, 4, 4, 30, 60)
    spec = O.Spec.of(inst)
    for _ in range(20):
        cm = (rng.random(spec.tb) < 0.5).astype(np.uint8)
        full = O.ruc_key(spec, cm, ruc, seed=1)
        for b in (1, 5, 12, 63, 64, 65, 100, 125):
            assert O.ruc_key(spec, cm, ruc, seed=1, bits=b) == (full >> (126 - b)) << (126 - b), b


@pytest.mark.parametrize("seed", range(4))
def test_hash_form_equals_exact_without_collisions(seed):
    """126-bit keyed sums do not collide on these sizes: the relaxed run caches the same
    languages as the exact one."""
    inst, cfg = synth.preset_instance("tiny", seed)
    assert int(inst.offsets[-1]) > 126
    ex = O.learn(inst, cfg["bound"])
    rx = O.learn(inst, cfg["bound"], ruc=O.RUC_HASH, ruc_seed=seed)
    assert rx.level_new == ex.level_new and rx.level_candidates == ex.level_candidates
    assert (rx.status, rx.cost, rx.first_index, rx.solution) == (ex.status, ex.cost, ex.first_index, ex.solution)


@pytest.mark.parametrize("ruc,bits", [(O.RUC_HASH, 6), (O.RUC_HASH, 10), (O.RUC_FKP, 0), (O.RUC_FKP, 9)])
@pytest.mark.parametrize("seed", range(3))
def test_relaxed_runs_are_sound(ruc, bits, seed):
    """False positives drop languages but never admit a wrong formula (Sec. 5): the
    result separates, costs at least the exact minimum, no two entries share a key, and
    no more languages are cached than there are keys."""
    inst, cfg = synth.preset_instance("tiny", seed)
    spec = O.Spec.of(inst)
    ex = O.learn(inst, cfg["bound"])
    run = O.Run(spec, cfg["bound"], ruc=ruc, ruc_seed=seed, ruc_bits=bits)
    rx = run.result()
    assert rx.status in (O.ST_OK, O.ST_NOT_FOUND)
    if rx.status == O.ST_OK:
        cm = O.eval_formula(spec, rx.solution)
        for t in range(inst.num_traces):
            assert bool(cm[int(inst.offsets[t])]) == (t < inst.num_pos)
        assert rx.cost >= ex.cost
    if bits:
        assert sum(rx.level_new) <= 1 << bits
    keys = set()
    n = 0
    for c in range(1, rx.levels_done + 1):
        for e in range(rx.level_new[c]):
            keys.add(O.ruc_key(spec, run.entry_cm(c, e), ruc, seed, bits))
            n += 1
    assert len(keys) == n

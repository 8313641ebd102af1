"""Seeded input generators checked against the recipes they state (CPU only).

The generators draw inputs for both the oracle and the GPU path, so a fault in them
would not show up as a parity failure.  Each check here uses code of its own: a
brute-force count of syntax trees, a textbook LTL evaluator (Sec. 2 semantics, one
position at a time), exact combinatorics and sampling statistics.
"""
import math
from collections import Counter
from itertools import combinations

import numpy as np
import pytest

from ltl_inputs import synth
from ltl_inputs.synth import ATOM, NOT, AND, OR, X, F, G, U


def _all_trees(size, props):
    """Every syntax tree with exactly `size` nodes, as nested tuples (brute force)."""
    if size == 1:
        return [("p", a) for a in range(props)]
    out = [(op, t) for op in ("!", "X", "F", "G") for t in _all_trees(size - 1, props)]
    for a in range(1, size - 1):
        for l in _all_trees(a, props):
            for r in _all_trees(size - 1 - a, props):
                out += [(op, l, r) for op in ("&", "|", "U")]
    return out


@pytest.mark.parametrize("props", [1, 2, 3])
def test_count_trees_matches_enumeration(props):
    S = synth.count_trees(6, props)
    for s in range(1, 7):
        assert S[s] == len(_all_trees(s, props)), (props, s)


def _tree_of(nodes, i=None):
    i = len(nodes) - 1 if i is None else i
    op, a, b = nodes[i]
    name = synth.OP_NAMES[op]
    if op == ATOM:
        return ("p", a)
    if op in (NOT, X, F, G):
        return (name, _tree_of(nodes, a))
    return (name, _tree_of(nodes, a), _tree_of(nodes, b))


def test_draw_formula_is_uniform_over_trees():
    # size 3 over one proposition: 16 unary chains and 3 binary trees, 19 in all
    trees = _all_trees(3, 1)
    assert len(trees) == 19
    rng = np.random.default_rng(7)
    n = 19 * 500
    hist = Counter(_tree_of(synth.draw_formula(rng, 3, 1)) for _ in range(n))
    assert set(hist) == set(trees)
    # expected 500 each, standard deviation about 22: 150 is about 7 deviations
    assert all(abs(c - 500) < 150 for c in hist.values()), hist


def _holds(nodes, i, tr, pos):
    """Textbook semantics at one position (strong X; F, G, U over [pos, |tr|))."""
    op, a, b = nodes[i]
    n = len(tr)
    if op == ATOM:
        return bool((int(tr[pos]) >> a) & 1)
    if op == NOT:
        return not _holds(nodes, a, tr, pos)
    if op == AND:
        return _holds(nodes, a, tr, pos) and _holds(nodes, b, tr, pos)
    if op == OR:
        return _holds(nodes, a, tr, pos) or _holds(nodes, b, tr, pos)
    if op == X:
        return pos + 1 < n and _holds(nodes, a, tr, pos + 1)
    if op == F:
        return any(_holds(nodes, a, tr, j) for j in range(pos, n))
    if op == G:
        return all(_holds(nodes, a, tr, j) for j in range(pos, n))
    assert op == U
    for j in range(pos, n):
        if _holds(nodes, b, tr, j):
            return True
        if not _holds(nodes, a, tr, j):
            return False
    return False


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_planted_instance_follows_its_recipe(seed):
    inst, cfg = synth.preset_instance("tiny", seed)
    k, lo, hi, A = cfg["k"], cfg["lo"], cfg["hi"], cfg["num_props"]
    assert inst.num_pos == k and inst.num_neg == k
    assert len(inst.planted) == cfg["size"]
    lens = inst.lengths
    assert lens.min() >= lo and lens.max() <= hi
    assert int(inst.letters.max()) < (1 << A)
    traces = [tuple(int(x) for x in inst.trace(t)) for t in range(inst.num_traces)]
    assert len(set(traces)) == len(traces)                    # distinct, classes disjoint
    root = len(inst.planted) - 1
    for t, tr in enumerate(traces):
        assert _holds(inst.planted, root, tr, 0) == (t < k), (seed, t)


def test_planted_labeler_agrees_with_textbook_semantics_everywhere():
    # every position of random traces, random formulas of every operator mix
    rng = np.random.default_rng(11)
    for trial in range(60):
        size = int(rng.integers(1, 8))
        A = int(rng.integers(1, 4))
        phi = synth.draw_formula(rng, size, A)
        n, Lmax = 16, 9
        lens = rng.integers(1, Lmax + 1, size=n)
        bits = rng.random((n, Lmax, A)) < 0.5
        bits &= (np.arange(Lmax)[None, :] < lens[:, None])[:, :, None]
        lab = synth._label_positions(phi, bits, lens)
        for r in range(n):
            tr = [int(sum(int(bits[r, j, p]) << p for p in range(A))) for j in range(lens[r])]
            for pos in range(lens[r]):
                assert lab[r, pos] == _holds(phi, len(phi) - 1, tr, pos), (trial, r, pos)
            assert not lab[r, lens[r]:].any()


@pytest.mark.parametrize("length,delta", [(3, 1), (4, 2), (5, 3)])
def test_hamming_instance_is_the_full_sphere(length, delta):
    inst = synth.hamming_instance(5, length, delta)
    assert inst.num_pos == 1 and inst.num_props == 2
    assert inst.num_neg == math.comb(2 * length, delta)
    p = [int(x) for x in inst.trace(0)]
    assert len(p) == length and max(p) < 4
    seen = set()
    for t in range(1, inst.num_traces):
        q = [int(x) for x in inst.trace(t)]
        assert len(q) == length
        assert sum(bin(a ^ b).count("1") for a, b in zip(p, q)) == delta
        seen.add(tuple(q))
    assert len(seen) == inst.num_neg


def test_poisson_arrivals():
    t = synth.poisson_arrivals(2, 20000, 10.0)
    assert t == synth.poisson_arrivals(2, 20000, 10.0)
    g = np.diff(np.concatenate([[0.0], t]))
    assert (g >= 0).all()
    # exponential gaps of mean 100 ms: the sample mean is within 3 % (4 standard errors),
    # and P(gap > mean) = 1/e
    assert abs(g.mean() - 100.0) < 3.0
    assert abs((g > 100.0).mean() - math.exp(-1)) < 0.015

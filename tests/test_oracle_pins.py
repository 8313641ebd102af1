"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

* the paper's worked examples (Sec. 4 and App. A), stored in tests/golden;
* an independent brute force over *all* syntax trees (no dedup, no canonical
  order) on tiny specifications: per-level counts of distinct languages and the
  minimal separating cost must agree with the oracle's exact enumerator;
* identities of finite-trace LTL (F = true U, G = not F not, De Morgan, X
  distributes over and/or, idempotence of F and G, the U expansion law, F as a
  disjunction of X^n, strong next at the last position);
* the two evaluation modes (quantifier clauses and backward expansion) agree
  exhaustively on all traces up to length 5 over two propositions;
* the planted formula bounds the minimal cost from above;
* OOM, inconsistency and invalid-input statuses.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import oracle as O
from ltl_inputs import synth
from ltl_text import (AND, ATOM, F, G, NOT, OR, U, X, all_traces, load_canonical_cases, load_paper_examples,
                      random_instance, single_trace_instance, trees_by_size)


# ---------------------------------------------------------------- worked examples

@pytest.mark.parametrize("mode", [O.MODE_QUANT, O.MODE_EXPAND])
def test_paper_worked_examples(mode):
    exs = load_paper_examples()
    assert len(exs) >= 20
    for ex in exs:
        inst = single_trace_instance(ex["letters"], len(ex["props"]))
        spec = O.Spec.of(inst)
        got = O.eval_formula(spec, ex["nodes"], mode).tolist()
        assert got == ex["bits"], (ex["name"], ex["cite"], got, ex["bits"])
        # the recursive textbook clauses agree position by position
        for i in range(len(ex["bits"])):
            assert O.holds(spec, 0, i, ex["nodes"]) == bool(ex["bits"][i]), (ex["name"], i)


# ---------------------------------------------------------------- exhaustive semantics

def _py_holds(tr, i, nodes, k):
    """Direct transcription of the satisfaction clauses, for cross-checking the C code."""
    n = len(tr)
    if i >= n:
        return False
    op, a, b = nodes[k]
    if op == ATOM:
        return bool((tr[i] >> a) & 1)
    if op == NOT:
        return not _py_holds(tr, i, nodes, a)
    if op == AND:
        return _py_holds(tr, i, nodes, a) and _py_holds(tr, i, nodes, b)
    if op == OR:
        return _py_holds(tr, i, nodes, a) or _py_holds(tr, i, nodes, b)
    if op == X:
        return _py_holds(tr, i + 1, nodes, a)
    if op == F:
        return any(_py_holds(tr, j, nodes, a) for j in range(i, n))
    if op == G:
        return all(_py_holds(tr, j, nodes, a) for j in range(i, n))
    if op == U:
        return any(_py_holds(tr, j, nodes, b) and all(_py_holds(tr, m, nodes, a) for m in range(i, j))
                   for j in range(i, n))
    raise ValueError(op)


def test_exhaustive_modes_agree():
    traces = list(all_traces(2, 5))
    assert len(traces) == 1364
    inst = synth.from_traces(traces, [], 2)
    spec = O.Spec.of(inst)
    trees = trees_by_size(5, 2)
    for s in range(1, 6):
        for nodes in trees[s]:
            q = O.eval_formula(spec, nodes, O.MODE_QUANT)
            e = O.eval_formula(spec, nodes, O.MODE_EXPAND)
            assert np.array_equal(q, e), nodes
    # and the C clauses agree with a Python transcription for all formulas up to size 3
    for s in range(1, 4):
        for nodes in trees[s]:
            q = O.eval_formula(spec, nodes, O.MODE_QUANT)
            k = 0
            for tr in traces:
                for i in range(len(tr)):
                    assert bool(q[k]) == _py_holds(tr, i, nodes, len(nodes) - 1), (nodes, tr, i)
                    k += 1


# ---------------------------------------------------------------- identities

def _cat(*parts):
    """Concatenate postfix formulas; returns (nodes, roots)."""
    nodes, roots = [], []
    for p in parts:
        off = len(nodes)
        for op, a, b in p:
            if op == ATOM:
                nodes.append((op, a, b))
            elif op in (AND, OR, U):
                nodes.append((op, a + off, b + off))
            else:
                nodes.append((op, a + off, 0))
        roots.append(len(nodes) - 1)
    return nodes, roots


def _un(op, f):
    return f + [(op, len(f) - 1, 0)]


def _bin(op, f, g):
    nodes, (ra, rb) = _cat(f, g)
    return nodes + [(op, ra, rb)]


def _true():
    return _bin(OR, [(ATOM, 0, 0)], _un(NOT, [(ATOM, 0, 0)]))


def test_identities_random():
    rng = np.random.default_rng(7)
    inst = random_instance(rng, 3, 40, 40, 1, 12)
    spec = O.Spec.of(inst)
    lens = inst.lengths
    last = np.zeros(inst.total_positions, dtype=bool)
    last[(inst.offsets[1:] - 1).astype(np.int64)] = True
    ev = lambda f: O.eval_formula(spec, f, O.MODE_QUANT)
    for trial in range(60):
        phi = synth.draw_formula(rng, int(rng.integers(1, 6)), 3)
        psi = synth.draw_formula(rng, int(rng.integers(1, 6)), 3)
        eq = lambda f, g: np.testing.assert_array_equal(ev(f), ev(g))
        eq(_un(F, phi), _bin(U, _true(), phi))                                     # F p == true U p
        eq(_un(G, phi), _un(NOT, _un(F, _un(NOT, phi))))                            # G p == !F!p
        eq(_un(NOT, _bin(AND, phi, psi)), _bin(OR, _un(NOT, phi), _un(NOT, psi)))   # De Morgan
        eq(_un(NOT, _bin(OR, phi, psi)), _bin(AND, _un(NOT, phi), _un(NOT, psi)))
        eq(_un(X, _bin(AND, phi, psi)), _bin(AND, _un(X, phi), _un(X, psi)))        # strong X distributes
        eq(_un(X, _bin(OR, phi, psi)), _bin(OR, _un(X, phi), _un(X, psi)))
        eq(_un(F, _un(F, phi)), _un(F, phi))                                        # FF = F (Sec. 4)
        eq(_un(G, _un(G, phi)), _un(G, phi))
        eq(_un(F, _bin(OR, phi, psi)), _bin(OR, _un(F, phi), _un(F, psi)))
        eq(_un(G, _bin(AND, phi, psi)), _bin(AND, _un(G, phi), _un(G, psi)))
        pu = _bin(U, phi, psi)                                                      # expansion law
        eq(pu, _bin(OR, psi, _bin(AND, phi, _un(X, pu))))
        eq(_bin(U, phi, phi), phi)                                                  # p U p == p
        disj = phi                                                                  # F p == OR_n X^n p
        xn = phi
        for _ in range(int(lens.max()) - 1):
            xn = _un(X, xn)
            disj = _bin(OR, disj, xn)
        eq(_un(F, phi), disj)
        a = ev(_un(NOT, _un(X, phi)))
        b = ev(_un(X, _un(NOT, phi)))
        assert np.all(a[last] == 1) and np.all(b[last] == 0)                        # strong next at the end
        assert np.array_equal(a[~last], b[~last])


# ---------------------------------------------------------------- brute force enumeration

def _bf_apply(op, A, B, inst):
    out = []
    for t in range(inst.num_traces):
        o, n = int(inst.offsets[t]), int(inst.offsets[t + 1] - inst.offsets[t])
        a = A[o:o + n]
        b = B[o:o + n] if B is not None else None
        for i in range(n):
            if op == NOT:
                v = not a[i]
            elif op == AND:
                v = a[i] and b[i]
            elif op == OR:
                v = a[i] or b[i]
            elif op == X:
                v = a[i + 1] if i + 1 < n else False
            elif op == F:
                v = any(a[i:])
            elif op == G:
                v = all(a[i:])
            else:
                v = any(b[j] and all(a[i:j]) for j in range(i, n))
            out.append(bool(v))
    return tuple(out)


def brute_force(inst, max_size, nnf=False, u_free=False):
    """All syntax trees up to max_size (no dedup): min size per language, min separating size.
    nnf: negation only directly above an atom; u_free: no U."""
    offs = inst.offsets.astype(np.int64)
    by_size = {1: []}
    for p in range(inst.num_props):
        by_size[1].append(tuple(bool((int(l) >> p) & 1) for l in inst.letters))
    for s in range(2, max_size + 1):
        cur = []
        for op in (NOT, X, F, G):
            if op == NOT and nnf and s - 1 != 1:
                continue
            cur += [_bf_apply(op, A, None, inst) for A in by_size[s - 1]]
        for op in ((AND, OR) if u_free else (AND, OR, U)):
            for a in range(1, s - 1):
                for A in by_size[a]:
                    for B in by_size[s - 1 - a]:
                        cur.append(_bf_apply(op, A, B, inst))
        by_size[s] = cur
    best = {}
    for s in range(1, max_size + 1):
        for cm in by_size[s]:
            best.setdefault(cm, s)
    counts = [0] * (max_size + 1)
    for s in best.values():
        counts[s] += 1
    cstar = None
    for s in range(1, max_size + 1):
        for cm in by_size[s]:
            if all(cm[offs[t]] for t in range(inst.num_pos)) and \
                    not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces)):
                cstar = s
                break
        if cstar:
            break
    return counts, cstar


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_levels_and_min_cost(seed):
    rng = np.random.default_rng(100 + seed)
    nprops = 1 + seed % 2
    inst = random_instance(rng, nprops, 2 + seed % 2, 2, 1, 4)
    max_size = 6 if nprops == 2 else 7
    counts, cstar = brute_force(inst, max_size)
    for mode in (O.MODE_QUANT, O.MODE_EXPAND):
        res = O.learn(inst, max_size, mode=mode)
        top = res.levels_done
        if cstar is None:
            assert res.status == O.ST_NOT_FOUND
        else:
            assert res.status == O.ST_OK and res.cost == cstar
        for c in range(1, top + 1):
            assert res.level_new[c] == counts[c], (c, res.level_new, counts)


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_levels_nnf_ufree(seed):
    # the operator sets of the experiments (Sec. 7): negation of atoms only, with and without U
    rng = np.random.default_rng(200 + seed)
    nprops = 1 + seed % 2
    inst = random_instance(rng, nprops, 2 + seed % 2, 2, 1, 4)
    max_size = 6 if nprops == 2 else 7
    for u_free in (False, True):
        counts, cstar = brute_force(inst, max_size, nnf=True, u_free=u_free)
        mask = (O.ALL_OPS & ~(1 << U) if u_free else O.ALL_OPS) | O.NNF
        res = O.learn(inst, max_size, op_mask=mask, mode=O.MODE_EXPAND)
        if cstar is None:
            assert res.status == O.ST_NOT_FOUND
        else:
            assert res.status == O.ST_OK and res.cost == cstar
        for c in range(1, res.levels_done + 1):
            assert res.level_new[c] == counts[c], (u_free, c, res.level_new, counts)


def test_nnf_solution_negates_atoms_only():
    # a spec whose unrestricted minimal formula negates a compound formula:
    # P = traces where p0 never holds, N = traces where it holds somewhere
    inst = synth.from_traces([[0, 0, 0], [0, 0]], [[0, 1, 0], [1, 0]], 1)
    full = O.learn(inst, 6)
    nnf = O.learn(inst, 6, op_mask=O.ALL_OPS | O.NNF)
    assert full.status == O.ST_OK and nnf.status == O.ST_OK
    assert full.cost == 3          # not F p0
    assert nnf.cost == 3           # G not p0
    nodes = nnf.solution
    for k, (op, a, b) in enumerate(nodes):
        if op == NOT:
            assert nodes[a][0] == 0, nodes     # the child of a negation is an atom


def test_bruteforce_no_solution_spec():
    # F p0 and X-structures cannot distinguish two traces that are identical: use
    # traces that differ only after position 0 in a way needing > 3 nodes
    inst = synth.from_traces([[1, 0, 0, 1]], [[1, 0, 1, 1]], 1)
    counts, cstar = brute_force(inst, 5)
    res = O.learn(inst, 5)
    assert (res.status == O.ST_OK) == (cstar is not None)
    if cstar is not None:
        assert res.cost == cstar
    for c in range(1, res.levels_done + 1):
        assert res.level_new[c] == counts[c]


# ---------------------------------------------------------------- planted workloads

@pytest.mark.parametrize("seed", range(16))
def test_planted_tiny_upper_bound_and_soundness(seed):
    inst, cfg = synth.preset_instance("tiny", seed)
    res = O.learn(inst, cfg["bound"])
    assert res.status == O.ST_OK
    assert res.cost <= cfg["size"]
    sol = res.solution
    assert len(sol) == res.cost                                   # unit costs: cost == size
    spec = O.Spec.of(inst)
    for t in range(inst.num_traces):
        assert O.holds(spec, t, 0, sol) == (t < inst.num_pos)
    # the planted formula separates too (labels come from it)
    for t in range(inst.num_traces):
        assert O.holds(spec, t, 0, inst.planted) == (t < inst.num_pos)


def test_threads_match_sequential():
    inst, cfg = synth.preset_instance("tiny", 0)
    a = O.learn(inst, 7, threads=1)
    b = O.learn(inst, 7, threads=4)
    assert (a.status, a.cost, a.level_new, a.level_candidates, a.first_index, a.solution) == \
           (b.status, b.cost, b.level_new, b.level_candidates, b.first_index, b.solution)


def test_candidate_counts_follow_canonical_order():
    inst, cfg = synth.preset_instance("tiny", 0)
    res = O.learn(inst, 7)
    E = res.level_new
    for c in range(2, res.levels_done + 1):
        x = c - 1
        expect = 4 * E[x]                                          # F, G, X, NOT
        for a in range(1, x):
            expect += E[a] * E[x - a]                              # U: ordered pairs
        for a in range(1, x // 2 + 1):
            b = x - a
            expect += 2 * (E[a] * E[b] if a < b else E[a] * (E[a] - 1) // 2)   # AND, OR
        assert res.level_candidates[c] == expect


def test_entry_formulas_reproduce_entry_matrices():
    inst, cfg = synth.preset_instance("tiny", 2)
    run = O.Run(O.Spec.of(inst), 5)
    res = run.result()
    for c in range(1, res.levels_done + 1):
        for i in range(0, res.level_new[c], max(1, res.level_new[c] // 7)):
            f = run.entry_formula(c, i)
            assert len(f) == c
            np.testing.assert_array_equal(O.eval_formula(run.spec, f), run.entry_cm(c, i))


# ---------------------------------------------------------------- canonical order (Sec. 3 listing)

@pytest.mark.parametrize("case", load_canonical_cases(), ids=lambda c: c["name"])
def test_canonical_order_first_solutions(case):
    """Which minimal formula is returned: hand-derived first solutions for each pair of
    neighbouring connectives in the Sec. 3 order, for the split order and for the pair
    order (tests/golden/canonical_order.txt)."""
    inst = case["inst"]
    res = O.learn(inst, case["expect_cost"] + 1, cost=case["cost"], op_mask=case["op_mask"])
    assert (res.status, res.cost) == (O.ST_OK, case["expect_cost"]), case["name"]
    assert res.first_index == case["expect_index"], (case["name"], res.first_index)
    assert res.solution == case["expect_formula"], (case["name"], res.solution)
    spec = O.Spec.of(inst)
    for t in range(inst.num_traces):
        assert O.holds(spec, t, 0, res.solution) == (t < inst.num_pos)


# ---------------------------------------------------------------- statuses

def test_oom_level_is_deterministic():
    inst, cfg = synth.preset_instance("tiny", 0)
    full = O.learn(inst, 7)
    E = full.level_new
    cum = np.cumsum(E)
    for cap in (1, 5, 20, int(cum[3])):
        res = O.learn(inst, 7, max_entries=cap)
        expect_level = int(np.argmax(cum > cap))
        if expect_level < full.cost:
            assert res.status == O.ST_EOOM and res.levels_done == expect_level
            assert res.level_new[:expect_level + 1] == E[:expect_level + 1]
        else:
            assert res.status == O.ST_OK


def test_invalid_and_inconsistent():
    inst = synth.from_traces([[1, 2]], [[1, 2]], 2)
    assert O.learn(inst, 4).status == O.ST_EINCONS
    inst = synth.from_traces([[1, 2], []], [[3]], 2)
    assert O.learn(inst, 4).status == O.ST_EINVAL
    inst = synth.from_traces([[4]], [[1]], 2)                  # letter bit beyond num_props
    assert O.learn(inst, 4).status == O.ST_EINVAL


def test_bound_and_atom_level():
    inst = synth.from_traces([[1, 0]], [[0, 1]], 1)
    res = O.learn(inst, 3)
    assert res.status == O.ST_OK and res.cost == 1 and res.solution == [(ATOM, 0, 0)]
    inst = synth.from_traces([[1, 0, 1]], [[1, 1, 1]], 1)      # needs X / G style formulas
    res1 = O.learn(inst, 1)
    assert res1.status == O.ST_NOT_FOUND and res1.levels_done == 1


# ---------------------------------------------------------------- overfitting (Sec. 2)

def _overfit_closed_cost(inst):
    """Unit costs: per trace of length n with m_i absent propositions at position i:
    sum_i (A + m_i + (A - 1)) literals and their ANDs, n ANDs joining a position to the rest,
    n - 1 X, and 6 for NOT X (p0 OR NOT p0); traces joined by |P| - 1 ORs."""
    A = inst.num_props
    total = 0
    for t in range(inst.num_pos):
        o, e = int(inst.offsets[t]), int(inst.offsets[t + 1])
        n = e - o
        absent = sum(A - bin(int(l) & ((1 << A) - 1)).count("1") for l in inst.letters[o:e])
        total += (2 * A - 1) * n + absent + n + (n - 1) + 6
    return total + inst.num_pos - 1


@pytest.mark.parametrize("seed", range(8))
def test_overfit_language_is_exactly_P(seed):
    rng = np.random.default_rng(300 + seed)
    nprops = 1 + seed % 3
    inst = random_instance(rng, nprops, 1 + seed % 3, 3, 1, 5)
    nodes, cost = O.overfit(inst)
    assert cost == _overfit_closed_cost(inst) == len(nodes)
    # on the specification: true at position 0 of every P trace, false on every N trace
    spec = O.Spec.of(inst)
    cm = O.eval_formula(spec, nodes, O.MODE_QUANT)
    offs = inst.offsets.astype(np.int64)
    assert all(cm[offs[t]] for t in range(inst.num_pos))
    assert not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces))
    # on traces next to P: one bit flipped, one letter longer or shorter -> outside P
    pos = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_pos)]
    near = []
    for tr in pos:
        for i in range(len(tr)):
            for k in range(nprops):
                v = list(tr); v[i] ^= 1 << k; near.append(v)
        near.append(tr + [0])
        if len(tr) > 1:
            near.append(tr[:-1])
    near = [v for v in near if v not in pos]
    probe = synth.from_traces(pos, near, nprops)
    cm2 = O.eval_formula(O.Spec.of(probe), nodes, O.MODE_EXPAND)
    o2 = probe.offsets.astype(np.int64)
    assert all(cm2[o2[t]] for t in range(probe.num_pos))
    assert not any(cm2[o2[t]] for t in range(probe.num_pos, probe.num_traces))


# ---------------------------------------------------------------- deterministic splitting (Sec. 6)

@pytest.mark.parametrize("seed", range(6))
def test_det_split_is_sound_and_plain_when_window_fits(seed):
    # planted specifications: every sub-specification is separated by the planted formula
    # (size 5), so each leaf stays cheap
    inst, cfg = synth.preset_instance("tiny", seed)
    offs = inst.offsets.astype(np.int64)
    trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
    P, N = trs[:inst.num_pos], trs[inst.num_pos:]
    for win in (3, 6, 12):
        st, f = O.det_split(P, N, inst.num_props, win)
        assert st == O.ST_OK and f is not None
        cm = O.eval_formula(O.Spec.of(inst), f, O.MODE_QUANT)
        assert all(cm[offs[t]] for t in range(inst.num_pos)), win
        assert not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces)), win
    # a window holding the whole specification: the learner's minimal formula
    st, f = O.det_split(P, N, inst.num_props, len(P) + len(N))
    assert f == O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND).solution


@pytest.mark.parametrize("seed", range(6))
def test_rand_split_is_sound_and_reproducible(seed):
    inst, cfg = synth.preset_instance("tiny", seed)
    offs = inst.offsets.astype(np.int64)
    trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
    P, N = trs[:inst.num_pos], trs[inst.num_pos:]
    for win, rs in ((4, 0), (8, 1), (12, 2)):
        st, f = O.rand_split(P, N, inst.num_props, win, seed=rs)
        assert st == O.ST_OK and f
        cm = O.eval_formula(O.Spec.of(inst), f, O.MODE_QUANT)
        assert all(cm[offs[t]] for t in range(inst.num_pos)), win
        assert not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces)), win
        assert O.rand_split(P, N, inst.num_props, win, seed=rs) == (st, f)
    st, f = O.rand_split(P, N, inst.num_props, len(P) + len(N))
    assert f == O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND).solution


# ---------------------------------------------------------------- random splitting's subsets

def test_splitmix64_published_outputs():
    # SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the first output of the generator
    # seeded with 0 is 0xE220A8397B1DCDAF and with 1234567 is 6457827717110365317 (the
    # values its reference implementation prints)
    assert O.splitmix64_output(0 + O.SPLITMIX_GAMMA) == 0xE220A8397B1DCDAF
    assert O.splitmix64_output(1234567 + O.SPLITMIX_GAMMA) == 6457827717110365317


def test_sample_subset():
    from collections import Counter
    a = O.sample_subset(3, 0, 100, 10)
    assert a == O.sample_subset(3, 0, 100, 10)                   # replayable
    assert a == sorted(set(a)) and len(a) == 10 and 0 <= a[0] and a[-1] < 100
    assert a != O.sample_subset(3, 1, 100, 10)                   # another stream, another subset
    assert O.sample_subset(3, 0, 5, 5) == [0, 1, 2, 3, 4]
    assert O.sample_subset(3, 0, 5, 9) == [0, 1, 2, 3, 4]
    # the k smallest draws of the stream, by brute force over the definition
    s0 = (7 << 32) + 4
    draws = [O.splitmix64_output(s0 + (i + 1) * O.SPLITMIX_GAMMA) for i in range(30)]
    assert O.sample_subset(7, 4, 30, 6) == sorted(sorted(range(30), key=lambda i: draws[i])[:6])
    # every element equally likely: k/n = 1/4 over 4000 draws of 5 of 20
    hits = Counter(x for c in range(4000) for x in O.sample_subset(1, c, 20, 5))
    assert all(abs(v - 1000) < 150 for v in hits.values()) and len(hits) == 20


def test_rand_split_halves_a_fitting_window_on_oom():
    # Sec. 6: randAux halves the window while the enumerator runs out of memory, also when
    # the whole specification fits the window (it is then drawn whole).  An entry cap of 12
    # makes the whole tiny specification run out of memory; the halved windows still
    # give a sound formula.
    inst, cfg = synth.preset_instance("tiny", 0)
    offs = inst.offsets.astype(np.int64)
    trs = [list(map(int, inst.letters[offs[t]:offs[t + 1]])) for t in range(inst.num_traces)]
    P, N = trs[:inst.num_pos], trs[inst.num_pos:]
    assert O.learn(inst, cfg["bound"], mode=O.MODE_EXPAND, max_entries=12).status == O.ST_EOOM
    st, f = O.rand_split(P, N, inst.num_props, len(P) + len(N), seed=0, max_entries=12)
    assert st == O.ST_OK and f
    cm = O.eval_formula(O.Spec.of(inst), f, O.MODE_QUANT)
    assert all(cm[offs[t]] for t in range(inst.num_pos))
    assert not any(cm[offs[t]] for t in range(inst.num_pos, inst.num_traces))

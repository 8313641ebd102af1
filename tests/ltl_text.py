"""Small helpers for tests: prefix-notation formulas, exhaustive trees, single-trace specs."""
from __future__ import annotations

import itertools
import os
from typing import Dict, List, Tuple

import numpy as np

from ltl_inputs import synth

ATOM, NOT, AND, OR, X, F, G, U = range(8)
_UN = {"!": NOT, "X": X, "F": F, "G": G}
_BIN = {"&": AND, "|": OR, "U": U}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse_prefix(text: str, props: List[str]):
    toks = text.split()
    nodes = []
    pos = 0

    def rec():
        nonlocal pos
        t = toks[pos]
        pos += 1
        if t in _UN:
            a = rec()
            nodes.append((_UN[t], a, 0))
        elif t in _BIN:
            a = rec()
            b = rec()
            nodes.append((_BIN[t], a, b))
        else:
            nodes.append((ATOM, props.index(t), 0))
        return len(nodes) - 1

    rec()
    assert pos == len(toks), text
    return nodes


def load_paper_examples():
    out = []
    with open(os.path.join(GOLDEN, "paper_examples.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, cite, props, trace, formula, bits = [x.strip() for x in line.split("|", 5)] if line.count("|") == 5 \
                else _split_example(line)
            props = props.split(",")
            letters = []
            for let in trace.split():
                m = 0
                if let != "-":
                    for p in let.split("+"):
                        m |= 1 << props.index(p)
                letters.append(m)
            out.append(dict(name=name, cite=cite, props=props, letters=letters,
                            nodes=parse_prefix(formula, props), bits=[int(c) for c in bits]))
    return out


def _split_example(line: str):
    # formulas may contain '|' (disjunction): split the first four fields and the last one
    parts = line.split("|")
    name, cite, props, trace = [p.strip() for p in parts[:4]]
    bits = parts[-1].strip()
    formula = "|".join(parts[4:-1]).strip()
    return name, cite, props, trace, formula, bits


def single_trace_instance(letters, num_props):
    return synth.from_traces([letters], [], num_props)


def all_traces(num_props: int, max_len: int):
    alpha = range(1 << num_props)
    for n in range(1, max_len + 1):
        for tr in itertools.product(alpha, repeat=n):
            yield list(tr)


def trees_by_size(max_size: int, num_props: int) -> Dict[int, List[list]]:
    """All syntax trees (postfix node lists) with exactly s nodes, s = 1..max_size."""
    T: Dict[int, List[list]] = {1: [[(ATOM, p, 0)] for p in range(num_props)]}

    def shift(nodes, k):
        return [(op, a + k if op != ATOM else a, (b + k) if op in (AND, OR, U) else b) for op, a, b in nodes]

    for s in range(2, max_size + 1):
        out = []
        for op in (NOT, X, F, G):
            for c in T[s - 1]:
                out.append(c + [(op, len(c) - 1, 0)])
        for op in (AND, OR, U):
            for a in range(1, s - 1):
                for l in T[a]:
                    for r in T[s - 1 - a]:
                        rr = shift(r, len(l))
                        out.append(l + rr + [(op, len(l) - 1, len(l) + len(rr) - 1)])
        T[s] = out
    return T


def random_instance(rng: np.random.Generator, num_props: int, npos: int, nneg: int, lo: int, hi: int,
                    p: float = 0.5):
    """Random distinct traces (no planted formula)."""
    seen = set()
    traces = []
    while len(traces) < npos + nneg:
        n = int(rng.integers(lo, hi + 1))
        tr = [int(x) for x in rng.integers(0, 1 << num_props, size=n)] if p == 0.5 else \
            [int(sum((1 << k) for k in range(num_props) if rng.random() < p)) for _ in range(n)]
        key = tuple(tr)
        if key in seen:
            continue
        seen.add(key)
        traces.append(tr)
    return synth.from_traces(traces[:npos], traces[npos:], num_props)


_CONN = {"F": F, "U": U, "G": G, "X": X, "&": AND, "|": OR, "!": NOT}


def _letters(text: str, props: List[str]):
    out = []
    for let in text.split():
        m = 0
        if let != "-":
            for p in let.split("+"):
                m |= 1 << props.index(p)
        out.append(m)
    return out


def load_canonical_cases():
    """Hand-derived first solutions (tests/golden/canonical_order.txt): per case the
    instance, op_mask, cost vector and the expected cost, first index and formula."""
    out = []
    with open(os.path.join(GOLDEN, "canonical_order.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, cite, props, conn, costs, P, N, cost, idx, formula = [x.strip() for x in line.split("::")]
            props = props.split(",")
            mask = 1
            for c in (_CONN.values() if conn == "all" else [_CONN[c] for c in conn.split(",")]):
                mask |= 1 << c
            cvec = [1] * 8
            if costs != "-":
                for item in costs.split(","):
                    k, v = item.split("=")
                    cvec[_CONN[k]] = int(v)
            pos = [_letters(t, props) for t in P.split(";")]
            neg = [_letters(t, props) for t in N.split(";")]
            out.append(dict(name=name, cite=cite, inst=synth.from_traces(pos, neg, len(props)), op_mask=mask,
                            cost=cvec, expect_cost=int(cost), expect_index=int(idx),
                            expect_formula=parse_prefix(formula, props)))
    return out

"""Seeded synthetic learning instances (specifications) for the LTL learner.

This module is the only code shared by the CPU oracle's tests and the GPU path's
tests/benchmarks.  It draws *inputs* only: traces, a planted formula and the
class split.  It contains no part of the enumerator (no characteristic
matrices, no operator bit tricks, no dedup, no separation search).  Labels are
assigned by evaluating the planted formula with a small numpy labeler written
for this module alone (backward recurrences over positions); a wrong label here
would only yield a different, still valid, specification for both sides.

Paper context:
  * A trace is a string over the powerset alphabet; a specification is a pair
    (P, N) of disjoint finite trace sets (Sec. 2, "Formal preliminaries").
  * BenchBase(Sigma, k, lo, hi) draws 2k uniform traces with lo <= |tr| <= hi
    (Sec. 7, "Benchmark construction").  The workloads here are planted-formula
    variants of it: letters are i.i.d. Bernoulli(p) per proposition and the
    class of a trace is tr |= phi_planted, so phi_planted separates (P, N) and
    the minimal cost is at most size(phi_planted).

Readings of the workload descriptions:
  * ranges "[lo, hi]" of the workload descriptions are inclusive;
  * the planted formula is uniform over syntax trees with exactly `size` nodes
    over {not, and, or, X, F, G, U} and atoms uniform over the propositions;
  * traces are resampled until each class holds k distinct traces; a trace
    already drawn (in either class) is rejected; after 10**6 draws without
    filling both classes the planted formula is redrawn from the next sub-seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

# Operator codes shared with include/ltl.h (LTL_ATOM ... LTL_U).
ATOM, NOT, AND, OR, X, F, G, U = range(8)
OP_NAMES = {ATOM: "p", NOT: "!", AND: "&", OR: "|", X: "X", F: "F", G: "G", U: "U"}
UNARY_OPS = (NOT, X, F, G)
BINARY_OPS = (AND, OR, U)


# --------------------------------------------------------------------------
# Formulas: postfix node lists [(op, a, b)], children referenced by node index;
# ATOM nodes carry the proposition index in `a`.
# --------------------------------------------------------------------------

def count_trees(size: int, num_props: int) -> List[int]:
    """S[s] = number of syntax trees with exactly s nodes (4 unary, 3 binary ops)."""
    S = [0] * (size + 1)
    if size >= 1:
        S[1] = num_props
    for s in range(2, size + 1):
        tot = 4 * S[s - 1]
        for a in range(1, s - 1):
            tot += 3 * S[a] * S[s - 1 - a]
        S[s] = tot
    return S


def draw_formula(rng: np.random.Generator, size: int, num_props: int) -> List[Tuple[int, int, int]]:
    """Uniform syntax tree with exactly `size` nodes, as a postfix node list."""
    S = count_trees(size, num_props)
    nodes: List[Tuple[int, int, int]] = []

    def uniform_below(n: int) -> int:
        # exact uniform integer in [0, n) for Python ints of any size
        if n <= (1 << 62):
            return int(rng.integers(0, n))
        while True:
            bits = n.bit_length()
            r = 0
            for _ in range((bits + 61) // 62):
                r = (r << 62) | int(rng.integers(0, 1 << 62))
            r &= (1 << bits) - 1
            if r < n:
                return r

    def build(s: int) -> int:
        r = uniform_below(S[s])
        if s == 1:
            nodes.append((ATOM, r, 0))
            return len(nodes) - 1
        for op in (NOT, X, F, G):
            if r < S[s - 1]:
                c = build(s - 1)
                nodes.append((op, c, 0))
                return len(nodes) - 1
            r -= S[s - 1]
        for op in (AND, OR, U):
            for a in range(1, s - 1):
                w = S[a] * S[s - 1 - a]
                if r < w:
                    ca = build(a)
                    cb = build(s - 1 - a)
                    nodes.append((op, ca, cb))
                    return len(nodes) - 1
                r -= w
        raise AssertionError("unreachable")

    build(size)
    return nodes


def formula_size(nodes: Sequence[Tuple[int, int, int]]) -> int:
    return len(nodes)


def formula_cost(nodes, cost: Sequence[int]) -> int:
    return sum(cost[op] for op, _, _ in nodes)


def formula_str(nodes, root: int | None = None) -> str:
    if root is None:
        root = len(nodes) - 1
    op, a, b = nodes[root]
    if op == ATOM:
        return f"p{a}"
    if op in (NOT, X, F, G):
        return f"{OP_NAMES[op]}({formula_str(nodes, a)})"
    return f"({formula_str(nodes, a)} {OP_NAMES[op]} {formula_str(nodes, b)})"


# --------------------------------------------------------------------------
# Labeler (input construction only): truth of a formula at every position of a
# batch of traces, via backward recurrences over positions.
# --------------------------------------------------------------------------

def _label_positions(nodes, bits: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """bits: bool [n, Lmax, A]; returns bool [n, Lmax] truth of the root."""
    n, Lmax, _ = bits.shape
    live = np.arange(Lmax)[None, :] < lens[:, None]
    vals = []
    for op, a, b in nodes:
        if op == ATOM:
            v = bits[:, :, a] & live
        elif op == NOT:
            v = ~vals[a] & live
        elif op == AND:
            v = vals[a] & vals[b]
        elif op == OR:
            v = vals[a] | vals[b]
        elif op == X:
            v = np.zeros_like(live)
            v[:, :-1] = vals[a][:, 1:]
            v &= live
        elif op == F:
            v = np.zeros_like(live)
            nxt = np.zeros(n, dtype=bool)
            for j in range(Lmax - 1, -1, -1):
                nxt = (vals[a][:, j] | nxt) & live[:, j]
                v[:, j] = nxt
        elif op == G:
            v = np.zeros_like(live)
            nxt = np.ones(n, dtype=bool)   # "always" holds vacuously after the end
            for j in range(Lmax - 1, -1, -1):
                cur = vals[a][:, j] & nxt
                nxt = np.where(live[:, j], cur, True)
                v[:, j] = cur & live[:, j]
        elif op == U:
            v = np.zeros_like(live)
            nxt = np.zeros(n, dtype=bool)
            for j in range(Lmax - 1, -1, -1):
                nxt = (vals[b][:, j] | (vals[a][:, j] & nxt)) & live[:, j]
                v[:, j] = nxt
        else:
            raise ValueError(op)
        vals.append(v)
    return vals[-1]


# --------------------------------------------------------------------------
# Instances
# --------------------------------------------------------------------------

@dataclass
class Instance:
    num_props: int
    letters: np.ndarray          # uint32, all letters of all traces, P first then N
    offsets: np.ndarray          # uint64, num_traces + 1
    num_pos: int
    num_neg: int
    planted: list = field(default_factory=list)   # postfix nodes (may be empty)
    seed: int = 0
    name: str = ""

    @property
    def num_traces(self) -> int:
        return self.num_pos + self.num_neg

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    @property
    def max_len(self) -> int:
        return int(self.lengths.max()) if self.num_traces else 0

    @property
    def total_positions(self) -> int:
        return int(self.offsets[-1])

    def trace(self, t: int) -> np.ndarray:
        return self.letters[int(self.offsets[t]):int(self.offsets[t + 1])]


def from_traces(pos: Sequence[Sequence[int]], neg: Sequence[Sequence[int]], num_props: int,
                name: str = "") -> Instance:
    """Instance from explicit traces; each trace is a list of letter bitmasks."""
    traces = [list(t) for t in pos] + [list(t) for t in neg]
    lens = [len(t) for t in traces]
    off = np.zeros(len(traces) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    flat = [x for t in traces for x in t]
    letters = np.asarray(flat, dtype=np.uint32)
    return Instance(num_props, letters, off, len(pos), len(neg), name=name)


def planted_instance(seed: int, num_props: int, k: int, lo: int, hi: int, p: float,
                     size: int, max_draws: int = 10 ** 6, batch: int = 4096,
                     name: str = "") -> Instance:
    """Planted-formula specification with k positive and k negative distinct traces.

    Traces are drawn in batches; a trace already drawn (in either class) is rejected.
    The planted formula is redrawn from the next sub-seed as soon as the class that
    fills slower cannot reach k within max_draws draws at its observed rate (checked
    after every batch once 16 384 traces were drawn), or when max_draws is reached.
    """
    attempt = 0
    weights = (1 << np.arange(num_props, dtype=np.uint32))
    while True:
        rng = np.random.default_rng([seed, attempt])
        phi = draw_formula(rng, size, num_props)
        pos: list = []
        neg: list = []
        seen = set()
        draws = 0
        n_pos_seen = n_neg_seen = 0
        feasible = True
        while (len(pos) < k or len(neg) < k) and draws < max_draws:
            nb = min(batch, max_draws - draws)
            lens = rng.integers(lo, hi + 1, size=nb)
            bits = rng.random((nb, hi, num_props), dtype=np.float32) < np.float32(p)
            live = np.arange(hi)[None, :] < lens[:, None]
            bits &= live[:, :, None]
            lab = _label_positions(phi, bits, lens)[:, 0]
            lets = (bits.astype(np.uint32) * weights[None, None, :]).sum(axis=2).astype(np.uint32)
            for i in range(nb):
                draws += 1
                cls = pos if lab[i] else neg
                if len(cls) >= k:
                    continue
                tr = lets[i, :lens[i]]
                key = tr.tobytes()
                if key in seen:
                    continue
                seen.add(key)
                cls.append(tr.copy())
                if len(pos) >= k and len(neg) >= k:
                    break
            n_pos_seen += int(lab.sum())
            n_neg_seen += int(nb - lab.sum())
            if draws >= 16384:
                rate = min(n_pos_seen, n_neg_seen) / draws
                if rate * max_draws < k:
                    feasible = False
                    break
        if feasible and len(pos) >= k and len(neg) >= k:
            break
        attempt += 1
    traces = pos + neg
    lens = np.array([len(t) for t in traces], dtype=np.uint64)
    off = np.zeros(len(traces) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    letters = np.concatenate(traces).astype(np.uint32)
    return Instance(num_props, letters, off, k, k, planted=phi, seed=seed, name=name)


# Workload presets: (props, k per class, len lo, len hi, Bernoulli p, planted size,
# cost bound, word bits).  "tiny", "scale" and "long" are the plain-method
# workloads.
PRESETS = {
    "tiny":  dict(num_props=2, k=16,   lo=4,  hi=8,   p=0.5, size=5,  bound=7,  word_bits=32),
    "scale": dict(num_props=3, k=1024, lo=16, hi=32,  p=0.5, size=9,  bound=11, word_bits=32),
    "long":  dict(num_props=5, k=4096, lo=64, hi=512, p=0.3, size=11, bound=13, word_bits=64),
}


def preset_instance(name: str, seed: int) -> Tuple[Instance, dict]:
    cfg = PRESETS[name]
    inst = planted_instance(seed, cfg["num_props"], cfg["k"], cfg["lo"], cfg["hi"], cfg["p"],
                            cfg["size"], name=f"{name}/{seed}")
    return inst, cfg


def hamming_instance(seed: int, length: int, delta: int) -> Instance:
    """Hamming(B, l, delta) over 2 propositions (2 bits per letter): P = {tr}, N = all
    traces of the same length at bit-Hamming distance delta (Sec. 7)."""
    from itertools import combinations
    rng = np.random.default_rng([seed, 0xA11])
    tr = rng.integers(0, 4, size=length).astype(np.uint32)
    negs = []
    for flips in combinations(range(2 * length), delta):
        t = tr.copy()
        for f in flips:
            t[f // 2] ^= np.uint32(1 << (f % 2))
        negs.append(t)
    return from_traces([tr.tolist()], [t.tolist() for t in negs], 2, name=f"hamming/{length}/{delta}/{seed}")


UNTIL_CHAINS = (64, 127, 128, 129, 255, 256, 257, 511)


def until_chain_instance(seed: int = 0, chains: Sequence[int] = UNTIL_CHAINS, extra: int = 4) -> Instance:
    """Traces over 2 propositions whose p0 U p1 needs long until-chains (App. B doubling
    across words of 64 positions).  For every d in `chains`:
      P gets p0^d p1       (p1 first at position d, p0 everywhere before it);
      N gets p0^d {}       (the same run with no p1 after it).
    P also gets one trace of runs p0^d p1 for the chains up to 129 back to back.  Both
    classes get `extra` random traces of length 64..512 with p0 ~ Bernoulli(0.95) and
    p1 ~ Bernoulli(0.03) (long runs of p0, rare p1), drawn from `seed`."""
    p0, p1 = 1, 2
    pos = [[p0] * d + [p1] for d in chains]
    neg = [[p0] * d + [0] for d in chains]
    runs = []
    for d in chains:
        if d <= 129:
            runs += [p0] * d + [p1]
    if runs:
        pos.append(runs)
    rng = np.random.default_rng([seed, 0xC4A1])
    seen = {tuple(t) for t in pos + neg}
    for cls in (pos, neg):
        added = 0
        while added < extra:
            n = int(rng.integers(64, 513))
            a = rng.random(n) < 0.95
            b = rng.random(n) < 0.03
            tr = tuple(int(x) for x in (a * p0 + b * p1))
            if tr in seen:
                continue
            seen.add(tr)
            cls.append(list(tr))
            added += 1
    return from_traces(pos, neg, 2, name=f"until-chains/{seed}")


def batched_jobs(master_seed: int = 0, njobs: int = 256):
    """The batched workload: independent jobs of uneven size.  Job j: propositions
    uniform in {2..5}, traces per class log-uniform in [16, 2048], lengths uniform in
    [8, 128], planted size uniform in [5, 10], Bernoulli(0.5) letters, cost bound =
    planted size + 2.  Returns a list of (Instance, bound)."""
    out = []
    for j in range(njobs):
        rng = np.random.default_rng([master_seed, 0xBA7C, j])
        A = int(rng.integers(2, 6))
        k = int(round(float(np.exp(rng.uniform(np.log(16), np.log(2048))))))
        size = int(rng.integers(5, 11))
        inst = planted_instance(1_000_003 * (master_seed + 1) + j, A, k, 8, 128, 0.5, size,
                                name=f"batched/{master_seed}/{j}")
        out.append((inst, size + 2))
    return out


def poisson_arrivals(seed: int, n: int, rate_per_s: float) -> List[float]:
    """Arrival times (milliseconds from 0, non-decreasing) of n jobs of a Poisson process of
    the given rate: exponential gaps from the stream `seed`."""
    rng = np.random.default_rng([seed, 0xA77])
    return [float(x) for x in np.cumsum(rng.exponential(1000.0 / rate_per_s, size=n))]

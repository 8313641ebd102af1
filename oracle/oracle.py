"""ctypes wrapper of the CPU oracle (oracle/ltl_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ltl_oracle.c")
LIB = os.environ.get("LTL_ORACLE_LIB") or os.path.join(HERE, "libltl_oracle.so")

ATOM, NOT, AND, OR, X, F, G, U = range(8)
MODE_QUANT, MODE_EXPAND = 0, 1
RUC_NONE, RUC_HASH, RUC_FKP = 0, 1, 2          # exact check; relaxed check of Sec. 5 (hash / FKP keys)
ST_OK, ST_NOT_FOUND, ST_EINVAL, ST_EINCONS, ST_EOOM = 0, 1, -1, -2, -4


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP for the candidate map)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Spec(C.Structure):
    _fields_ = [("num_props", C.c_int32), ("num_pos", C.c_int32), ("num_neg", C.c_int32),
                ("pad_", C.c_int32), ("letters", C.c_void_p), ("offsets", C.c_void_p)]


class _Node(C.Structure):
    _fields_ = [("op", C.c_int32), ("a", C.c_int32), ("b", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("LTL_ORACLE_LIB") and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = C.CDLL(LIB)
        L.oracle_holds.argtypes = [C.POINTER(_Spec), C.c_int, C.c_int64, C.POINTER(_Node), C.c_int]
        L.oracle_holds.restype = C.c_int
        L.oracle_apply.argtypes = [C.POINTER(_Spec), C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.oracle_apply.restype = C.c_int
        L.oracle_eval_formula.argtypes = [C.POINTER(_Spec), C.POINTER(_Node), C.c_int, C.c_int, C.c_void_p]
        L.oracle_eval_formula.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(_Spec), C.POINTER(C.c_int32), C.c_uint32, C.c_int, C.c_int,
                                 C.c_int, C.c_int64]
        L.oracle_run.restype = C.c_void_p
        L.oracle_run_relaxed.argtypes = [C.POINTER(_Spec), C.POINTER(C.c_int32), C.c_uint32, C.c_int, C.c_int,
                                         C.c_int, C.c_int64, C.c_int, C.c_uint64, C.c_int]
        L.oracle_run_relaxed.restype = C.c_void_p
        L.oracle_ruc_key.argtypes = [C.POINTER(_Spec), C.c_void_p, C.c_int, C.c_uint64, C.c_int, C.c_void_p]
        L.oracle_ruc_key.restype = C.c_int
        L.oracle_fkp_k.argtypes = [C.POINTER(_Spec), C.c_void_p]
        L.oracle_fkp_k.restype = C.c_int
        L.oracle_free.argtypes = [C.c_void_p]
        for name, rt in [("oracle_status", C.c_int), ("oracle_found_cost", C.c_int),
                         ("oracle_levels_done", C.c_int), ("oracle_first_index", C.c_int64)]:
            getattr(L, name).argtypes = [C.c_void_p]
            getattr(L, name).restype = rt
        for name, rt in [("oracle_level_new", C.c_int64), ("oracle_level_candidates", C.c_int64),
                         ("oracle_level_seconds", C.c_double)]:
            getattr(L, name).argtypes = [C.c_void_p, C.c_int]
            getattr(L, name).restype = rt
        L.oracle_entry_formula.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.POINTER(_Node), C.c_int]
        L.oracle_entry_formula.restype = C.c_int
        L.oracle_solution_formula.argtypes = [C.c_void_p, C.POINTER(_Node), C.c_int]
        L.oracle_solution_formula.restype = C.c_int
        L.oracle_entry_cm.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p]
        L.oracle_entry_cm.restype = C.c_int
        _lib = L
    return _lib


class Spec:
    """Keeps the numpy buffers alive for the C structure."""

    def __init__(self, num_props: int, letters: np.ndarray, offsets: np.ndarray, num_pos: int, num_neg: int):
        self.letters = np.ascontiguousarray(letters, dtype=np.uint32)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.num_pos, self.num_neg, self.num_props = num_pos, num_neg, num_props
        self.c = _Spec(num_props, num_pos, num_neg, 0, self.letters.ctypes.data if self.letters.size else None,
                       self.offsets.ctypes.data)
        self.tb = int(self.offsets[-1])

    @classmethod
    def of(cls, inst) -> "Spec":
        return cls(inst.num_props, inst.letters, inst.offsets, inst.num_pos, inst.num_neg)


def _nodes(nodes) -> "C.Array":
    arr = (_Node * len(nodes))()
    for k, (op, a, b) in enumerate(nodes):
        arr[k].op, arr[k].a, arr[k].b = op, a, b
    return arr


def holds(spec: Spec, t: int, i: int, nodes) -> bool:
    r = lib().oracle_holds(C.byref(spec.c), t, i, _nodes(nodes), len(nodes))
    assert r >= 0
    return bool(r)


def eval_formula(spec: Spec, nodes, mode: int = MODE_QUANT) -> np.ndarray:
    out = np.zeros(spec.tb, dtype=np.uint8)
    assert lib().oracle_eval_formula(C.byref(spec.c), _nodes(nodes), len(nodes), mode, out.ctypes.data) == 0
    return out


def apply(spec: Spec, op: int, a: np.ndarray, b: Optional[np.ndarray] = None, mode: int = MODE_QUANT) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    out = np.zeros(spec.tb, dtype=np.uint8)
    bp = None
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.uint8)
        bp = b.ctypes.data
    assert lib().oracle_apply(C.byref(spec.c), op, a.ctypes.data, bp, mode, out.ctypes.data) == 0
    return out


UNIT_COST = [1] * 8
ALL_OPS = 0xFF
NNF = 1 << 8                                   # op_mask flag: negation of atoms only
U_FREE_NNF = (ALL_OPS & ~(1 << U)) | NNF       # the operator set of the experiments of Sec. 7


@dataclass
class Result:
    status: int
    cost: int
    levels_done: int
    level_new: List[int]          # index = cost level
    level_candidates: List[int]
    level_seconds: List[float]
    first_index: int
    solution: Optional[list] = None
    run: Optional["Run"] = field(default=None, repr=False)


class Run:
    def __init__(self, spec: Spec, bound: int, cost=UNIT_COST, op_mask: int = ALL_OPS, mode: int = MODE_QUANT,
                 threads: int = 1, max_entries: int = 0, ruc: int = RUC_NONE, ruc_seed: int = 0, ruc_bits: int = 0):
        self.spec = spec
        self.bound = bound
        c = (C.c_int32 * 8)(*cost)
        self.h = lib().oracle_run_relaxed(C.byref(spec.c), c, op_mask, bound, mode, threads, max_entries,
                                          ruc, ruc_seed, ruc_bits)
        assert self.h

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_free(self.h)
            self.h = None

    def result(self) -> Result:
        L = lib()
        st = L.oracle_status(self.h)
        done = L.oracle_levels_done(self.h)
        E = [max(0, L.oracle_level_new(self.h, c)) for c in range(self.bound + 1)]
        Cc = [max(0, L.oracle_level_candidates(self.h, c)) for c in range(self.bound + 1)]
        S = [L.oracle_level_seconds(self.h, c) for c in range(self.bound + 1)]
        sol = None
        if st == ST_OK:
            buf = (_Node * 4096)()
            n = L.oracle_solution_formula(self.h, buf, 4096)
            sol = [(buf[k].op, buf[k].a, buf[k].b) for k in range(n)]
        return Result(st, L.oracle_found_cost(self.h), done, E, Cc, S, L.oracle_first_index(self.h), sol, self)

    def entry_formula(self, c: int, i: int):
        buf = (_Node * 4096)()
        n = lib().oracle_entry_formula(self.h, c, i, buf, 4096)
        assert n > 0
        return [(buf[k].op, buf[k].a, buf[k].b) for k in range(n)]

    def entry_cm(self, c: int, i: int) -> np.ndarray:
        out = np.zeros(self.spec.tb, dtype=np.uint8)
        assert lib().oracle_entry_cm(self.h, c, i, out.ctypes.data) == 0
        return out


def overfit(inst, cost=UNIT_COST):
    """The overfitting formula of (P, N), written out from its definition (Sec. 2):
      overfit(letter)   = AND over the propositions of p_k (present) or NOT p_k (absent)
      overfit(a . tr)   = overfit(a) AND X overfit(tr)      (tr non-empty)
      overfit(a)        = overfit(a) AND NOT X true           (a the last letter: the trace ends)
      overfit(P, N)     = OR over tr in P of overfit(tr);  true = p0 OR NOT p0
    (The printed base case puts the end marker under one more X, which with the strong X of
    Sec. 2 would describe traces one letter longer; the reading above gives L = P.)
    Returns (postfix nodes (op, a, b) with the root last, cost)."""
    nodes = []

    def emit(op, a=0, b=0):
        nodes.append((op, a, b))
        return len(nodes) - 1

    def letter(bits):
        root = None
        for k in range(inst.num_props):
            lit = emit(ATOM, k)
            if not (bits >> k) & 1:
                lit = emit(NOT, lit)
            root = lit if root is None else emit(AND, root, lit)
        return root

    def trace(letters):
        head = letter(int(letters[0]))
        if len(letters) == 1:
            tru = emit(OR, emit(ATOM, 0), emit(NOT, emit(ATOM, 0)))
            return emit(AND, head, emit(NOT, emit(X, tru)))
        return emit(AND, head, emit(X, trace(letters[1:])))

    root = None
    for t in range(inst.num_pos):
        o, e = int(inst.offsets[t]), int(inst.offsets[t + 1])
        f = trace(inst.letters[o:e])
        root = f if root is None else emit(OR, root, f)
    return nodes, sum(cost[op] for op, _, _ in nodes)


def formula_tree(nodes, k=None):
    """Postfix nodes -> nested tuples (shape only), for comparing encodings of one formula."""
    k = len(nodes) - 1 if k is None else k
    op, a, b = nodes[k]
    if op == ATOM:
        return (ATOM, a)
    if op in (NOT, X, F, G):
        return (op, formula_tree(nodes, a))
    return (op, formula_tree(nodes, a), formula_tree(nodes, b))


def det_split(pos, neg, num_props: int, win: int, cost=UNIT_COST, op_mask: int = ALL_OPS, max_entries: int = 0,
              threads: int = 1):
    """Deterministic splitting (Sec. 6), with the learner of Sec. 3 at the leaves: enumerate
    the levels below the cost of overfitting, else the overfitting formula.  L = the traces
    accepted by both formulas of the first pair (their conjunction), R24.  Returns
    (status, postfix nodes or None)."""
    from ltl_inputs import synth

    def accepted(nodes, traces):
        if not traces:
            return []
        sp = Spec.of(synth.from_traces(traces, [], num_props))
        cm = eval_formula(sp, nodes, MODE_EXPAND)
        starts = sp.offsets[:-1].astype(np.int64)
        return [bool(cm[o]) for o in starts]

    def leaf(P, N):
        inst = synth.from_traces(P, N, num_props)
        of_nodes, of_cost = overfit(inst, cost)
        r = learn(inst, min(of_cost - 1, 63), cost, op_mask, MODE_EXPAND, threads, max_entries)
        if r.status == ST_OK:
            return ST_OK, r.solution
        if r.status == ST_NOT_FOUND:
            return ST_OK, of_nodes
        return r.status, None

    def combine(op, f, g):
        shift = len(f)
        moved = []
        for o, a, b in g:
            if o == ATOM:
                moved.append((o, a, b))
            elif o in (AND, OR, U):
                moved.append((o, a + shift, b + shift))
            else:
                moved.append((o, a + shift, b))
        return f + moved + [(op, shift - 1, shift + len(g) - 1)]

    def split(P, N, w):
        if len(P) == 0:
            return ST_OK, None
        if len(P) + len(N) <= w or max(len(P), len(N)) <= 1:
            return leaf(P, N)
        P1, P2 = P[:len(P) // 2], P[len(P) // 2:]
        N1, N2 = N[:len(N) // 2], N[len(N) // 2:]
        st, f11 = split(P1, N1, w)
        f12 = None
        if st == ST_OK and f11 is not None:
            left = [n for n, ok in zip(N2, accepted(f11, N2)) if ok]
            if left:
                st, f12 = split(P1, left, w)
        first = None if f11 is None else (f11 if f12 is None else combine(AND, f11, f12))
        f21 = f22 = None
        if st == ST_OK:
            P2r = P2 if first is None else [p for p, ok in zip(P2, accepted(first, P2)) if not ok]
            st, f21 = split(P2r, N1, w)
            if st == ST_OK and f21 is not None:
                left = [n for n, ok in zip(N2, accepted(f21, N2)) if ok]
                if left:
                    st, f22 = split(P2r, left, w)
        if st == ST_EOOM:
            return (ST_EOOM, None) if w <= 1 else split(P, N, w // 2)
        if st != ST_OK:
            return st, None
        second = None if f21 is None else (f21 if f22 is None else combine(AND, f21, f22))
        if first is None:
            return ST_OK, second
        return ST_OK, first if second is None else combine(OR, first, second)

    return split(list(pos), list(neg), win)


_M64 = (1 << 64) - 1
SPLITMIX_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_output(state: int) -> int:
    """SplitMix64's output function (Steele, Lea and Flood, "Fast splittable pseudorandom
    number generators", OOPSLA 2014): the generator adds GAMMA to its state and returns
    this mix of the new state."""
    z = state & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sample_subset(seed: int, stream: int, n: int, k: int):
    """The random subset of random splitting: k of range(n), those whose draws from the
    SplitMix64 sequence started at state seed * 2^32 + stream are smallest (draw i is the
    output after i + 1 steps), in increasing order; all of range(n) when k >= n."""
    if k >= n:
        return list(range(n))
    s0 = (seed << 32) + stream
    keys = [splitmix64_output(s0 + (i + 1) * SPLITMIX_GAMMA) for i in range(n)]
    return sorted(sorted(range(n), key=lambda i: (keys[i], i))[:k])


def rand_split(pos, neg, num_props: int, win: int, seed: int = 0, cost=UNIT_COST, op_mask: int = ALL_OPS,
               max_entries: int = 0, threads: int = 1):
    """Random splitting (Sec. 6) with the learner of Sec. 3 at the leaves.  The q-th random
    sub-specification of the recursion (in call order) draws its positives from stream 2q
    and its negatives from stream 2q + 1 of `sample_subset`.  randAux halves the window
    while the learner runs out of memory; a specification that fits the window is drawn
    whole.  Returns (status, nodes or None); an empty node list stands for "true" (no
    negative trace left to reject)."""
    from ltl_inputs import synth
    draws = [0]

    def accepted(nodes, traces):
        if not traces:
            return []
        sp = Spec.of(synth.from_traces(traces, [], num_props))
        cm = eval_formula(sp, nodes, MODE_EXPAND)
        return [bool(cm[o]) for o in sp.offsets[:-1].astype(np.int64)]

    def leaf(P, N):
        inst = synth.from_traces(P, N, num_props)
        of_nodes, of_cost = overfit(inst, cost)
        r = learn(inst, min(of_cost - 1, 63), cost, op_mask, MODE_EXPAND, threads, max_entries)
        if r.status == ST_OK:
            return ST_OK, r.solution
        if r.status == ST_NOT_FOUND:
            return ST_OK, of_nodes
        return r.status, None

    def conj(f, g):
        if f is None or g is None:
            return None
        if len(g) == 0:
            return f
        if len(f) == 0:
            return g
        k = len(f)
        return f + [(o, a if o == ATOM else a + k, b + k if o in (AND, OR, U) else b) for o, a, b in g] + \
            [(AND, k - 1, k + len(g) - 1)]

    def disj(f, g):
        if f is None:
            return g
        if g is None:
            return f
        k = len(f)
        return f + [(o, a if o == ATOM else a + k, b + k if o in (AND, OR, U) else b) for o, a, b in g] + \
            [(OR, k - 1, k + len(g) - 1)]

    def split(P, N):
        if len(P) == 0:
            return ST_OK, None
        if len(N) == 0:
            return ST_OK, []
        w = win
        while True:
            if w < 2:
                return ST_EOOM, None
            total = min(w, len(P) + len(N))
            kp = min(len(P), (total + 1) // 2)
            kn = min(len(N), total - kp)
            kp = min(len(P), total - kn)
            call = draws[0]
            draws[0] += 1
            P0 = [P[i] for i in sample_subset(seed, 2 * call, len(P), kp)]
            N0 = [N[i] for i in sample_subset(seed, 2 * call + 1, len(N), kn)]
            st, f11 = leaf(P0, N0)
            if st != ST_EOOM:
                break
            w //= 2
        if st != ST_OK:
            return st, None
        aP, aN = accepted(f11, P), accepted(f11, N)
        P_in = [p for p, a in zip(P, aP) if a]
        P_out = [p for p, a in zip(P, aP) if not a]
        N_in = [n for n, a in zip(N, aN) if a]
        N_out = [n for n, a in zip(N, aN) if not a]
        st, f12 = split(P_in, N_in)
        if st != ST_OK:
            return st, None
        st, f21 = split(P_out, N_out)
        if st != ST_OK:
            return st, None
        st, f22 = split(P_out, N_in)
        if st != ST_OK:
            return st, None
        return ST_OK, disj(conj(f11, f12), conj(f21, f22))

    return split(list(pos), list(neg))


def learn(inst, bound: int, cost=UNIT_COST, op_mask: int = ALL_OPS, mode: int = MODE_QUANT, threads: int = 1,
          max_entries: int = 0, ruc: int = RUC_NONE, ruc_seed: int = 0, ruc_bits: int = 0) -> Result:
    spec = Spec.of(inst)
    run = Run(spec, bound, cost, op_mask, mode, threads, max_entries, ruc, ruc_seed, ruc_bits)
    return run.result()


def ruc_key(spec: Spec, cm: np.ndarray, kind: int, seed: int = 0, bits: int = 0) -> int:
    """The 126-bit key of the relaxed check (Sec. 5) of one matrix (one byte per
    position, trace-major), as an integer whose bit 125 is the key's first bit."""
    cm = np.ascontiguousarray(cm, dtype=np.uint8)
    out = (C.c_uint64 * 2)()
    assert lib().oracle_ruc_key(C.byref(spec.c), cm.ctypes.data, kind, seed, bits, out) == 0
    return (out[0] << 62) | (out[1] >> 2)


def fkp_prefixes(spec: Spec):
    """FKP (Sec. 7): (k, positions kept per trace); k = 0 when the whole matrix fits 126 bits."""
    m = np.zeros(spec.num_pos + spec.num_neg, dtype=np.int64)
    k = lib().oracle_fkp_k(C.byref(spec.c), m.ctypes.data)
    assert k >= 0
    return k, [int(x) for x in m]


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB, file=sys.stderr)

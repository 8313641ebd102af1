"""Python binding of the gfx950 LTL learner library (libltl.so, C-ABI in include/ltl.h).

Argument marshalling only: every step of the learner runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  Importing works
without a GPU; creating a context needs the built library and a HIP device and
raises otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; LTL_LIBRARY names another build of the same sources
LIB_PATH = os.environ.get("LTL_LIBRARY") or os.path.join(PKG, "libltl.so")

LTL_OK, LTL_NOT_FOUND = 0, 1
LTL_E_INVAL, LTL_E_INCONSISTENT, LTL_E_TOO_LONG, LTL_E_OOM, LTL_E_DEVICE, LTL_E_STATE = -1, -2, -3, -4, -5, -6
LTL_E_BUFFER = -7
ATOM, NOT, AND, OR, X, F, G, U = range(8)
CTX_U_CARRY, CTX_TIMING, CTX_TIMING_LEVEL, CTX_RUC, CTX_U_DOUBLING = 0x1, 0x2, 0x4, 0x8, 0x10
CTX_LDS_TILES = 0x20   # binary tiles of whole-row levels stage 8 x 8 groups of child words in LDS
CTX_RUC_FKP = 0x40     # with CTX_RUC: first-k-percent keys (Sec. 7) instead of the keyed sums
CTX_ONE_STREAM = 0x80  # no second stream for the U class of whole-row levels
BATCH_BIG_ALONE = 0x100    # batch flag: whole-row levels of different lanes take turns
BATCH_SHARED_BUDGET = 0x200   # batch flag: one memory budget, regions sized per job
SPEC_DEVICE = 0x1
MAX_LEVELS, MAX_NODES, K_KINDS = 64, 64, 6
NO_SOLUTION = (1 << 64) - 1
KERNEL_KINDS = ("eval", "verify", "materialize", "compact", "fallback", "intake")

# every symbol include/ltl.h declares
EXPORTS = ("ltl_ctx_create", "ltl_ctx_destroy", "ltl_learn", "ltl_learn_batch", "ltl_batch_create", "ltl_batch_run",
           "ltl_batch_destroy", "ltl_job_create", "ltl_eval_level",
           "ltl_job_result", "ltl_job_formula", "ltl_job_dump_cm", "ltl_job_get_info", "ltl_job_destroy",
           "ltl_status_str", "ltl_overfit", "ltl_batch_serve", "ltl_holds", "ltl_det_split", "ltl_rand_split",
           "ltl_learn_noalloc", "ltl_batch_get_stats", "ltl_autotune")


class LTLError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _status_str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class CtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_uint32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64), ("stream", C.c_void_p), ("hash_slots_log2", C.c_uint32),
                ("word_bits", C.c_uint32), ("fp_bits", C.c_uint32), ("split_tiles", C.c_uint32),
                ("max_entries", C.c_uint64), ("ruc_seed", C.c_uint64), ("ruc_key_bits", C.c_uint32),
                ("reserved", C.c_uint32)]


class Spec(C.Structure):
    _fields_ = [("num_props", C.c_uint32), ("num_pos", C.c_uint32), ("num_neg", C.c_uint32),
                ("flags", C.c_uint32), ("letters", C.c_void_p), ("offsets", C.c_void_p)]


class OpSet(C.Structure):
    _fields_ = [("op_mask", C.c_uint32), ("cost", C.c_uint32 * 8)]


class Node(C.Structure):
    _fields_ = [("op", C.c_uint32), ("a", C.c_uint32), ("b", C.c_uint32)]


class BatchOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_uint32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64), ("lanes", C.c_uint32), ("hash_slots_log2", C.c_uint32),
                ("word_bits", C.c_uint32), ("fp_bits", C.c_uint32), ("max_entries", C.c_uint64),
                ("split_tiles", C.c_uint32), ("reserved", C.c_uint32)]


TUNE_CONFIGS = 5


class Tuning(C.Structure):
    _fields_ = [("tried", C.c_uint32), ("best", C.c_uint32), ("flags", C.c_uint32 * TUNE_CONFIGS),
                ("split_tiles", C.c_uint32 * TUNE_CONFIGS), ("ms", C.c_double * TUNE_CONFIGS)]


class BatchJob(C.Structure):
    _fields_ = [("spec", Spec), ("ops", OpSet), ("cost_bound", C.c_uint32), ("reserved", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("cost", C.c_uint32), ("levels_done", C.c_uint32),
                ("num_nodes", C.c_uint32), ("nodes", Node * MAX_NODES), ("solution_index", C.c_uint64),
                ("level_new", C.c_uint64 * MAX_LEVELS), ("level_candidates", C.c_uint64 * MAX_LEVELS),
                ("level_ms", C.c_double * MAX_LEVELS), ("colliders", C.c_uint64),
                ("kernel_ms", C.c_double * K_KINDS), ("kernel_launches", C.c_uint32 * K_KINDS),
                ("pad", C.c_uint32), ("level_bytes", C.c_uint64 * MAX_LEVELS)]


class BatchStats(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("peak_bytes", C.c_uint64), ("admissions", C.c_uint32),
                ("reruns", C.c_uint32), ("max_in_flight", C.c_uint32), ("pad", C.c_uint32),
                ("region_bytes_total", C.c_uint64)]


class LevelStats(C.Structure):
    _fields_ = [("cost", C.c_uint32), ("stored", C.c_uint32), ("candidates", C.c_uint64),
                ("new_entries", C.c_uint64), ("first_solution", C.c_uint64), ("colliders", C.c_uint64),
                ("kernel_ms", C.c_double), ("alg_bytes", C.c_uint64)]


class JobInfo(C.Structure):
    _fields_ = [("word_bits", C.c_uint32), ("rows", C.c_uint32), ("cm_bytes", C.c_uint64),
                ("total_positions", C.c_uint64), ("hash_slots_log2", C.c_uint32), ("doubling_steps", C.c_uint32),
                ("arena_bytes", C.c_uint64), ("max_entries", C.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libltl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_2402_12373_amd.build`")
    L = C.CDLL(path)
    P = C.POINTER
    L.ltl_ctx_create.argtypes = [P(CtxOpts), P(C.c_void_p)]
    L.ltl_ctx_create.restype = C.c_int
    L.ltl_ctx_destroy.argtypes = [C.c_void_p]
    L.ltl_ctx_destroy.restype = None
    L.ltl_learn.argtypes = [C.c_void_p, P(Spec), P(OpSet), C.c_uint32, P(Result)]
    L.ltl_learn.restype = C.c_int
    L.ltl_learn_batch.argtypes = [P(BatchOpts), P(BatchJob), C.c_uint32, P(Result), P(C.c_double)]
    L.ltl_learn_batch.restype = C.c_int
    L.ltl_batch_create.argtypes = [P(BatchOpts), P(C.c_void_p)]
    L.ltl_batch_create.restype = C.c_int
    L.ltl_batch_run.argtypes = [C.c_void_p, P(BatchJob), C.c_uint32, P(Result), P(C.c_double)]
    L.ltl_batch_run.restype = C.c_int
    L.ltl_batch_serve.argtypes = [C.c_void_p, P(BatchJob), C.c_uint32, P(C.c_double), P(Result), P(C.c_double)]
    L.ltl_batch_serve.restype = C.c_int
    L.ltl_autotune.argtypes = [C.c_void_p, P(Spec), P(OpSet), C.c_uint32, P(Tuning)]
    L.ltl_autotune.restype = C.c_int
    L.ltl_batch_get_stats.argtypes = [C.c_void_p, P(BatchStats)]
    L.ltl_batch_get_stats.restype = C.c_int
    L.ltl_batch_destroy.argtypes = [C.c_void_p]
    L.ltl_batch_destroy.restype = None
    L.ltl_job_create.argtypes = [C.c_void_p, P(Spec), P(OpSet), C.c_uint32, P(C.c_void_p)]
    L.ltl_job_create.restype = C.c_int
    L.ltl_eval_level.argtypes = [C.c_void_p, C.c_uint32, P(LevelStats)]
    L.ltl_eval_level.restype = C.c_int
    L.ltl_job_result.argtypes = [C.c_void_p, P(Result)]
    L.ltl_job_result.restype = C.c_int
    L.ltl_overfit.argtypes = [P(Spec), P(OpSet), P(Node), C.c_uint32, P(C.c_uint32), P(C.c_uint64)]
    L.ltl_overfit.restype = C.c_int
    L.ltl_learn_noalloc.argtypes = [C.c_int32, C.c_void_p, P(Spec), P(OpSet), C.c_uint32, P(Result)]
    L.ltl_learn_noalloc.restype = C.c_int
    L.ltl_holds.argtypes = [C.c_void_p, P(Spec), P(Node), C.c_uint32, C.c_void_p]
    L.ltl_holds.restype = C.c_int
    L.ltl_det_split.argtypes = [C.c_void_p, P(Spec), P(OpSet), C.c_uint32, P(Node), C.c_uint32, P(C.c_uint32)]
    L.ltl_det_split.restype = C.c_int
    L.ltl_rand_split.argtypes = [C.c_void_p, P(Spec), P(OpSet), C.c_uint32, C.c_uint64, P(Node), C.c_uint32,
                                 P(C.c_uint32)]
    L.ltl_rand_split.restype = C.c_int
    L.ltl_job_formula.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, P(Node), C.c_uint32, P(C.c_uint32)]
    L.ltl_job_formula.restype = C.c_int
    L.ltl_job_dump_cm.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, C.c_void_p, C.c_uint64]
    L.ltl_job_dump_cm.restype = C.c_int
    L.ltl_job_get_info.argtypes = [C.c_void_p, P(JobInfo)]
    L.ltl_job_get_info.restype = C.c_int
    L.ltl_job_destroy.argtypes = [C.c_void_p]
    L.ltl_job_destroy.restype = None
    L.ltl_status_str.argtypes = [C.c_int]
    L.ltl_status_str.restype = C.c_char_p
    _lib = L
    return L


def _status_str(st: int) -> str:
    try:
        return load_library().ltl_status_str(st).decode()
    except Exception:
        return f"status {st}"


OPS_NNF = 1 << 8      # op_mask flag (LTL_OPS_NNF): negation of atoms only


def opset(cost: Optional[Sequence[int]] = None, ops: Optional[Sequence[int]] = None, nnf: bool = False) -> OpSet:
    """Operator set: `ops` lists the enabled connectives (default all; ATOM is always
    enabled) or is a raw op_mask integer (LTL_OPS_NNF included), `cost` their costs
    (default 1), `nnf` restricts negation to atoms."""
    o = OpSet()
    if isinstance(ops, int):
        mask = ops
    else:
        mask = 0
        for op in (ops if ops is not None else range(8)):
            mask |= 1 << op
    o.op_mask = mask | 1 | (OPS_NNF if nnf else 0)
    for k in range(8):
        o.cost[k] = (cost[k] if cost is not None else 1)
    return o


@dataclass
class LearnResult:
    status: int
    cost: int
    levels_done: int
    level_new: List[int]
    level_candidates: List[int]
    level_ms: List[float]
    solution: Optional[list]
    solution_index: Optional[int]
    colliders: int
    kernel_ms: dict = field(default_factory=dict)
    kernel_launches: dict = field(default_factory=dict)
    level_bytes: List[int] = field(default_factory=list)

    @property
    def candidates(self) -> int:
        return int(sum(self.level_candidates))


def _convert(r: Result) -> LearnResult:
    done = int(r.levels_done)
    sol = [(int(r.nodes[k].op), int(r.nodes[k].a), int(r.nodes[k].b)) for k in range(r.num_nodes)] \
        if r.status == LTL_OK else None
    return LearnResult(int(r.status), int(r.cost), done,
                       [int(r.level_new[c]) for c in range(done + 1)],
                       [int(r.level_candidates[c]) for c in range(done + 1)],
                       [float(r.level_ms[c]) for c in range(done + 1)], sol,
                       None if r.solution_index == NO_SOLUTION else int(r.solution_index), int(r.colliders),
                       {KERNEL_KINDS[k]: float(r.kernel_ms[k]) for k in range(K_KINDS)},
                       {KERNEL_KINDS[k]: int(r.kernel_launches[k]) for k in range(K_KINDS)},
                       [int(r.level_bytes[c]) for c in range(done + 1)])


class SpecBuffers:
    """Host (numpy) or device (torch) buffers behind an ltl_spec."""

    def __init__(self, inst, device_tensors=None):
        self.inst = inst
        self.c = Spec()
        self.c.num_props = inst.num_props
        self.c.num_pos = inst.num_pos
        self.c.num_neg = inst.num_neg
        if device_tensors is None:
            self.letters = np.ascontiguousarray(inst.letters, dtype=np.uint32)
            self.offsets = np.ascontiguousarray(inst.offsets, dtype=np.uint64)
            self.c.flags = 0
            self.c.letters = self.letters.ctypes.data
            self.c.offsets = self.offsets.ctypes.data
        else:
            self.letters, self.offsets = device_tensors
            self.c.flags = SPEC_DEVICE
            self.c.letters = self.letters.data_ptr()
            self.c.offsets = self.offsets.data_ptr()


def overfit(inst, cost=None, ops=None):
    """The overfitting formula of (P, N) (Sec. 2) and its cost: (postfix nodes (op, a, b), root
    last; cost under the operator set).  Host-only, no device."""
    L = load_library()
    sb = SpecBuffers(inst)
    o = opset(cost, ops)
    n, c = C.c_uint32(0), C.c_uint64(0)
    st = L.ltl_overfit(C.byref(sb.c), C.byref(o), None, 0, C.byref(n), C.byref(c))
    if st not in (LTL_OK, LTL_E_OOM):
        raise LTLError(st, "ltl_overfit")
    buf = (Node * max(1, n.value))()
    st = L.ltl_overfit(C.byref(sb.c), C.byref(o), buf, n.value, C.byref(n), C.byref(c))
    if st != LTL_OK:
        raise LTLError(st, "ltl_overfit")
    return [(int(buf[k].op), int(buf[k].a), int(buf[k].b)) for k in range(n.value)], int(c.value)


def learn_complete(ctx: "Context", inst_or_spec, inst=None, cost=None, ops=None) -> LearnResult:
    """The learner of Sec. 3: enumerate the cost levels below the cost of overfitting; if no
    formula there separates (P, N), the overfitting formula is the answer (status LTL_OK,
    solution_index None).  `inst` gives the host traces when inst_or_spec is a device spec.
    When the cost of overfitting exceeds the level range, the enumeration stops at the last
    level and its result is returned as is (no claim of minimality for a fallback)."""
    host = inst if inst is not None else inst_or_spec
    nodes, co = overfit(host, cost, ops)
    bound = min(co - 1, MAX_LEVELS - 1)
    r = ctx.learn(inst_or_spec, bound, cost, ops)
    if r.status == LTL_NOT_FOUND and bound == co - 1:
        return replace(r, status=LTL_OK, cost=co, solution=nodes, solution_index=None)
    return r


NOALLOC_SCRATCH_BYTES = 64 << 20     # LTL_NOALLOC_SCRATCH_BYTES
NOALLOC_SLOTS_LOG2 = 18              # LTL_NOALLOC_SLOTS_LOG2


def learn_noalloc(inst_or_spec, bound: int, device: int = 0, stream=None, cost=None, ops=None) -> LearnResult:
    """ltl_learn_noalloc: learning on the library's fixed device scratch array (no workspace,
    no allocation); `stream` is a torch stream (default: the device's current stream)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the LTL learner has no CPU path")
    L = load_library()
    spec = inst_or_spec if isinstance(inst_or_spec, SpecBuffers) else SpecBuffers(inst_or_spec)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    r = Result()
    L.ltl_learn_noalloc(device, stream.cuda_stream, C.byref(spec.c), C.byref(opset(cost, ops)), bound, C.byref(r))
    return _convert(r)


def spec_to_device(inst, device="cuda"):
    """Copies an instance's letters/offsets to device tensors (inputs resident in HBM)."""
    import torch
    letters = torch.from_numpy(np.ascontiguousarray(inst.letters, dtype=np.uint32).view(np.int32)).to(device)
    offsets = torch.from_numpy(np.ascontiguousarray(inst.offsets, dtype=np.uint64).view(np.int64)).to(device)
    return SpecBuffers(inst, (letters, offsets))


class Context:
    """An ltl_ctx over a torch-allocated device workspace."""

    def __init__(self, workspace_bytes: int = 1 << 30, device: int = 0, flags: int = 0, hash_slots_log2: int = 0,
                 word_bits: int = 0, fp_bits: int = 0, max_entries: int = 0, stream=None, workspace=None,
                 split_tiles: int = 0, ruc_seed: int = 0, ruc_key_bits: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the LTL learner has no CPU path")
        L = load_library()
        self.L = L
        self.device = device
        if workspace is None:
            workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.workspace = workspace
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        o = CtxOpts()
        o.device = device
        o.flags = flags
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
        o.stream = stream.cuda_stream
        o.hash_slots_log2 = hash_slots_log2
        o.word_bits = word_bits
        o.fp_bits = fp_bits
        o.split_tiles = split_tiles
        o.max_entries = max_entries
        o.ruc_seed = ruc_seed
        o.ruc_key_bits = ruc_key_bits
        self.opts = o
        h = C.c_void_p()
        st = L.ltl_ctx_create(C.byref(o), C.byref(h))
        if st != LTL_OK:
            raise LTLError(st, "ltl_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.ltl_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def learn(self, inst_or_spec, bound: int, cost=None, ops=None) -> LearnResult:
        spec = inst_or_spec if isinstance(inst_or_spec, SpecBuffers) else SpecBuffers(inst_or_spec)
        r = Result()
        self.L.ltl_learn(self.h, C.byref(spec.c), C.byref(opset(cost, ops)), bound, C.byref(r))
        return _convert(r)

    def autotune(self, inst_or_spec, bound: int, cost=None, ops=None):
        """ltl_autotune: times the job under each tile shape / level schedule; returns
        (best (flags, split_tiles), [(flags, split_tiles, ms), ...])."""
        spec = inst_or_spec if isinstance(inst_or_spec, SpecBuffers) else SpecBuffers(inst_or_spec)
        t = Tuning()
        st = self.L.ltl_autotune(self.h, C.byref(spec.c), C.byref(opset(cost, ops)), bound, C.byref(t))
        if st != LTL_OK:
            raise LTLError(st, "ltl_autotune")
        rows = [(int(t.flags[k]), int(t.split_tiles[k]), float(t.ms[k])) for k in range(t.tried)]
        return rows[t.best][:2], rows

    def job(self, inst_or_spec, bound: int, cost=None, ops=None) -> "Job":
        return Job(self, inst_or_spec, bound, cost, ops)


class Job:
    """Level-by-level interface (ltl_job_create / ltl_eval_level / ...)."""

    def __init__(self, ctx: Context, inst_or_spec, bound: int, cost=None, ops=None):
        self.ctx = ctx
        self.L = ctx.L
        self.spec = inst_or_spec if isinstance(inst_or_spec, SpecBuffers) else SpecBuffers(inst_or_spec)
        self.bound = bound
        h = C.c_void_p()
        st = self.L.ltl_job_create(ctx.h, C.byref(self.spec.c), C.byref(opset(cost, ops)), bound, C.byref(h))
        if st != LTL_OK:
            raise LTLError(st, "ltl_job_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.ltl_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval_level(self, cost: int) -> LevelStats:
        s = LevelStats()
        st = self.L.ltl_eval_level(self.h, cost, C.byref(s))
        if st != LTL_OK:
            raise LTLError(st, f"ltl_eval_level({cost})")
        return s

    def result(self) -> LearnResult:
        r = Result()
        self.L.ltl_job_result(self.h, C.byref(r))
        return _convert(r)

    def formula(self, cost: int, entry: int):
        buf = (Node * MAX_NODES)()
        n = C.c_uint32()
        st = self.L.ltl_job_formula(self.h, cost, entry, buf, MAX_NODES, C.byref(n))
        if st != LTL_OK:
            raise LTLError(st, "ltl_job_formula")
        return [(int(buf[k].op), int(buf[k].a), int(buf[k].b)) for k in range(n.value)]

    def dump_cm(self, cost: int, entry: int) -> np.ndarray:
        tb = int(self.spec.inst.total_positions)
        out = np.zeros(tb, dtype=np.uint8)
        st = self.L.ltl_job_dump_cm(self.h, cost, entry, out.ctypes.data, tb)
        if st != LTL_OK:
            raise LTLError(st, "ltl_job_dump_cm")
        return out

    def info(self) -> JobInfo:
        i = JobInfo()
        st = self.L.ltl_job_get_info(self.h, C.byref(i))
        if st != LTL_OK:
            raise LTLError(st, "ltl_job_get_info")
        return i


def _batch_opts(workspace, lanes, device, flags, hash_slots_log2, word_bits, fp_bits, max_entries, split_tiles=0):
    o = BatchOpts()
    o.device, o.flags, o.workspace = device, flags, workspace.data_ptr()
    o.workspace_bytes = workspace.numel()
    o.lanes, o.hash_slots_log2, o.word_bits, o.fp_bits, o.max_entries = lanes, hash_slots_log2, word_bits, \
        fp_bits, max_entries
    o.split_tiles = split_tiles
    return o


def _batch_jobs(specs, bounds, cost, ops):
    bufs = [s if isinstance(s, SpecBuffers) else SpecBuffers(s) for s in specs]
    jobs = (BatchJob * len(bufs))()
    for i, b in enumerate(bufs):
        jobs[i].spec = b.c
        jobs[i].ops = opset(cost, ops)
        jobs[i].cost_bound = int(bounds[i])
    return jobs, bufs


class Batch:
    """A batch executor (ltl_batch_create): `lanes` contexts, each with its own stream,
    workspace slice and hash table, kept across runs."""

    def __init__(self, lanes: int = 4, workspace_bytes: int = 8 << 30, device: int = 0, flags: int = 0,
                 hash_slots_log2: int = 0, word_bits: int = 0, fp_bits: int = 0, max_entries: int = 0,
                 workspace=None, split_tiles: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the LTL learner has no CPU path")
        self._L = load_library()
        if workspace is None:
            workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.workspace = workspace
        self.lanes = lanes
        o = _batch_opts(workspace, lanes, device, flags, hash_slots_log2, word_bits, fp_bits, max_entries,
                        split_tiles)
        h = C.c_void_p()
        torch.cuda.synchronize()
        st = self._L.ltl_batch_create(C.byref(o), C.byref(h))
        if st != LTL_OK:
            raise LTLError(st, "ltl_batch_create")
        self._h = h

    def run(self, specs, bounds, cost=None, ops=None):
        """Runs the jobs; returns (results, durations_ms, completion_ms)."""
        jobs, bufs = _batch_jobs(specs, bounds, cost, ops)
        n = len(bufs)
        res = (Result * n)()
        ms = (C.c_double * (2 * n))()
        st = self._L.ltl_batch_run(self._h, jobs, n, res, ms)
        if st != LTL_OK:
            raise LTLError(st, "ltl_batch_run")
        return [_convert(res[i]) for i in range(n)], [ms[2 * i] for i in range(n)], [ms[2 * i + 1] for i in range(n)]

    def serve(self, specs, bounds, arrival_ms, cost=None, ops=None):
        """Serving (ltl_batch_serve): job i arrives arrival_ms[i] after the call begins; returns
        (results, durations_ms, completion_ms); latency = completion - arrival."""
        jobs, bufs = _batch_jobs(specs, bounds, cost, ops)
        n = len(bufs)
        res = (Result * n)()
        ms = (C.c_double * (2 * n))()
        arr = (C.c_double * max(1, n))(*[float(a) for a in arrival_ms])
        st = self._L.ltl_batch_serve(self._h, jobs, n, arr, res, ms)
        if st != LTL_OK:
            raise LTLError(st, "ltl_batch_serve")
        return [_convert(res[i]) for i in range(n)], [ms[2 * i] for i in range(n)], [ms[2 * i + 1] for i in range(n)]

    def stats(self) -> BatchStats:
        """Memory accounting of the last run (shared-budget batches)."""
        st = BatchStats()
        rc = self._L.ltl_batch_get_stats(self._h, C.byref(st))
        if rc != LTL_OK:
            raise LTLError(rc, "ltl_batch_get_stats")
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._L.ltl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def learn_batch(specs, bounds, lanes: int = 8, workspace_bytes: int = 8 << 30, device: int = 0, flags: int = 0,
                hash_slots_log2: int = 0, word_bits: int = 0, fp_bits: int = 0, max_entries: int = 0,
                cost=None, ops=None, workspace=None):
    """Runs many jobs, `lanes` at a time (ltl_learn_batch).  Returns (results, durations_ms, completion_ms)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the LTL learner has no CPU path")
    L = load_library()
    if workspace is None:
        workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
    o = _batch_opts(workspace, lanes, device, flags, hash_slots_log2, word_bits, fp_bits, max_entries)
    jobs, bufs = _batch_jobs(specs, bounds, cost, ops)
    n = len(bufs)
    res = (Result * n)()
    ms = (C.c_double * (2 * n))()
    torch.cuda.synchronize()
    st = L.ltl_learn_batch(C.byref(o), jobs, n, res, ms)
    if st != LTL_OK:
        raise LTLError(st, "ltl_learn_batch")
    return [_convert(res[i]) for i in range(n)], [ms[2 * i] for i in range(n)], [ms[2 * i + 1] for i in range(n)]


# ---------------------------------------------------------------- formulas on traces, divide and conquer (Sec. 6)

class _Traces:
    """An (instance-like) host specification built from explicit traces."""

    def __init__(self, pos, neg, num_props: int):
        traces = [list(t) for t in pos] + [list(t) for t in neg]
        self.num_props, self.num_pos, self.num_neg = int(num_props), len(pos), len(neg)
        self.offsets = np.zeros(len(traces) + 1, dtype=np.uint64)
        self.offsets[1:] = np.cumsum([len(t) for t in traces], dtype=np.uint64)
        self.letters = np.asarray([x for t in traces for x in t], dtype=np.uint32)
        self.total_positions = int(self.offsets[-1])


def _node_array(nodes):
    arr = (Node * max(1, len(nodes)))()
    for k, (op, a, b) in enumerate(nodes):
        arr[k].op, arr[k].a, arr[k].b = op, a, b
    return arr


def holds(ctx: "Context", traces, nodes, num_props: int) -> np.ndarray:
    """tr |= phi for each trace (ltl_holds: the formula evaluated on the device)."""
    if not traces:
        return np.zeros(0, dtype=bool)
    sb = SpecBuffers(_Traces(traces, [], num_props))
    out = np.zeros(len(traces), dtype=np.uint8)
    st = ctx.L.ltl_holds(ctx.h, C.byref(sb.c), _node_array(nodes), len(nodes), out.ctypes.data)
    if st != LTL_OK:
        raise LTLError(st, "ltl_holds")
    return out.astype(bool)


def _split_call(fn, args, what):
    n = C.c_uint32(0)
    cap = 1024
    while True:
        buf = (Node * cap)()
        st = fn(*args, buf, cap, C.byref(n))
        if st == LTL_E_BUFFER:
            cap = int(n.value)
            continue
        if st != LTL_OK:
            return st, None
        return LTL_OK, [(int(buf[k].op), int(buf[k].a), int(buf[k].b)) for k in range(n.value)]


def det_split(ctx: "Context", pos, neg, num_props: int, win: int, cost=None, ops=None):
    """Deterministic splitting (ltl_det_split, Sec. 6).  Returns (status, postfix nodes or
    None): LTL_OK and a sound formula, or LTL_E_OOM when even a window of 1 runs out of
    memory."""
    sb = SpecBuffers(_Traces(pos, neg, num_props))
    o = opset(cost, ops)
    return _split_call(ctx.L.ltl_det_split, (ctx.h, C.byref(sb.c), C.byref(o), int(win)), "ltl_det_split")


def rand_split(ctx: "Context", pos, neg, num_props: int, win: int, seed: int = 0, cost=None, ops=None):
    """Random splitting (ltl_rand_split, Sec. 6) with the library's counter-based subset
    draws from `seed`.  Returns (status, postfix nodes or None)."""
    sb = SpecBuffers(_Traces(pos, neg, num_props))
    o = opset(cost, ops)
    return _split_call(ctx.L.ltl_rand_split, (ctx.h, C.byref(sb.c), C.byref(o), int(win), int(seed)),
                       "ltl_rand_split")

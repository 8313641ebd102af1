"""CPU-side checks of the C-ABI: the library exports every declared symbol and the
Python binding's structures have the header's layout (size and field offsets)."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltl.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ltl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2402_12373_amd import build, ltl
    if not os.path.exists(ltl.LIB_PATH):
        build.build(verbose=False)
    return ltl.LIB_PATH


def test_library_exports_every_declared_symbol(lib_path):
    from paper_2402_12373_amd import ltl
    names = _declared_functions()
    assert set(names) == set(ltl.EXPORTS), (names, ltl.EXPORTS)
    lib = C.CDLL(lib_path)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_binding_struct_layout_matches_header(tmp_path):
    from paper_2402_12373_amd import ltl
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ltl.h"
#define S(t) printf(#t " %zu\n", sizeof(t))
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f))
int main(void) {
  S(ltl_ctx_opts); O(ltl_ctx_opts, workspace); O(ltl_ctx_opts, stream); O(ltl_ctx_opts, max_entries);
  S(ltl_spec); O(ltl_spec, letters); O(ltl_spec, offsets);
  S(ltl_opset); S(ltl_node);
  S(ltl_result); O(ltl_result, solution_index); O(ltl_result, level_new); O(ltl_result, level_ms);
  O(ltl_result, colliders); O(ltl_result, kernel_ms); O(ltl_result, kernel_launches);
  O(ltl_result, level_bytes);
  S(ltl_level_stats); O(ltl_level_stats, kernel_ms); O(ltl_level_stats, alg_bytes);
  S(ltl_job_info); O(ltl_job_info, arena_bytes);
  S(ltl_batch_opts); O(ltl_batch_opts, workspace); O(ltl_batch_opts, lanes); O(ltl_batch_opts, max_entries);
  S(ltl_batch_job); O(ltl_batch_job, ops); O(ltl_batch_job, cost_bound);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    m = {"ltl_ctx_opts": ltl.CtxOpts, "ltl_spec": ltl.Spec, "ltl_opset": ltl.OpSet, "ltl_node": ltl.Node,
         "ltl_result": ltl.Result, "ltl_level_stats": ltl.LevelStats, "ltl_job_info": ltl.JobInfo,
         "ltl_batch_opts": ltl.BatchOpts, "ltl_batch_job": ltl.BatchJob}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(m[t], f).offset == int(val), key
        else:
            assert C.sizeof(m[key]) == int(val), key


def test_context_without_gpu_fails_loudly():
    import torch
    from paper_2402_12373_amd import ltl
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        ltl.Context(workspace_bytes=1 << 24)


def test_generator_is_deterministic():
    from ltl_inputs import synth
    a, _ = synth.preset_instance("tiny", 5)
    b, _ = synth.preset_instance("tiny", 5)
    assert (a.letters == b.letters).all() and (a.offsets == b.offsets).all() and a.planted == b.planted
    c, _ = synth.preset_instance("tiny", 6)
    assert not ((len(a.letters) == len(c.letters)) and (a.letters == c.letters).all())
    # planted formulas have exactly the requested size and are drawn over the full grammar
    S = synth.count_trees(5, 2)
    assert S[1:] == [2, 8, 44, 272, 1808]
    assert synth.count_trees(9, 3)[9] == 17176746


def test_hamming_generator_size():
    from ltl_inputs import synth
    inst = synth.hamming_instance(0, 12, 2)
    assert inst.num_pos == 1 and inst.num_neg == 24 * 23 // 2


def test_overfit_matches_oracle_and_rejects_bad_sets():
    """ltl_overfit is host-only: the library's formula equals the oracle's (same tree, same
    cost) for random specifications and operator costs; NNF and sets without X are refused."""
    from oracle import oracle as O
    from ltl_text import random_instance
    from paper_2402_12373_amd import ltl
    rng = np.random.default_rng(17)
    for seed in range(12):
        inst = random_instance(rng, 1 + seed % 3, 1 + seed % 4, 2, 1, 6)
        cost = [int(c) for c in rng.integers(1, 4, size=8)]
        nodes, c = ltl.overfit(inst, cost=cost)
        onodes, oc = O.overfit(inst, cost)
        assert c == oc and O.formula_tree(nodes) == O.formula_tree(onodes), seed
    inst = random_instance(rng, 2, 2, 2, 1, 4)
    for ops in (0xFF | ltl.OPS_NNF, 0xFF & ~(1 << ltl.X), 0xFF & ~(1 << ltl.OR)):
        with pytest.raises(ltl.LTLError):
            ltl.overfit(inst, ops=ops)

"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of oracle/ltl_oracle.c with one plausible mistake (weak
next, wrong G base case, off-by-one in the U or F quantifier, no dedup, swapped
classes in the separation check, an extra X at the last position, negation of
compound formulae in negation normal form).  It is
compiled on the CPU and the pin tests are run against it; every mutant must
make at least one pin fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ltl_oracle.c")

MUTANTS = {
    "weak_next": ("case O_X:   for (int64_t i = 0; i < len; ++i) R[i] = (i + 1 < len) ? A[i + 1] : 0; break;",
                  "case O_X:   for (int64_t i = 0; i < len; ++i) R[i] = (i + 1 < len) ? A[i + 1] : 1; break;"),
    "G_base": ("int nxt = 1;                /* base", "int nxt = 0;                /* base"),
    "F_strict": ("for (int64_t j = i; j < len; ++j) if (A[j]) { v = 1; break; }",
                 "for (int64_t j = i + 1; j < len; ++j) if (A[j]) { v = 1; break; }"),
    "U_inclusive": ("for (int64_t m = i; m < j; ++m) if (!A[m]) { ok = 0; break; }",
                    "for (int64_t m = i; m <= j; ++m) if (!A[m]) { ok = 0; break; }"),
    "no_dedup": ("if (!map_contains(r, pk, B->hv[k])) {", "if (1) {"),
    "swapped_classes": ("if (t < s->num_pos ? !v : v) return 0;", "if (t < s->num_pos ? v : !v) return 0;"),
    "U_expand_no_phi": ("nxt = B[i] || (A[i] && nxt);", "nxt = B[i] || nxt;"),
    "nnf_ignored": ("if (op == O_NOT && (r->op_mask & O_NNF) && x != r->cost[O_ATOM]) continue;", ";"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    msrc = tmp_path / "mut.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(msrc)])
    env = dict(os.environ, LTL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-k", "worked or bruteforce_levels or planted_tiny or identities or exhaustive"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

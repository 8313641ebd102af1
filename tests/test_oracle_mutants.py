"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of oracle/ltl_oracle.c with one plausible mistake (weak
next, wrong G base case, off-by-one in the U or F quantifier, no dedup, swapped
classes in the separation check, an extra X at the last position, negation of
compound formulae in negation normal form, neighbouring connectives of the Sec. 3
order exchanged, splits or pairs enumerated in the other order).  It is
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
    "no_dedup": ("if (!map_contains(r, pk, key, B->hv[k])) {", "if (1) {"),
    "swapped_classes": ("if (t < s->num_pos ? !v : v) return 0;", "if (t < s->num_pos ? v : !v) return 0;"),
    "U_expand_no_phi": ("nxt = B[i] || (A[i] && nxt);", "nxt = B[i] || nxt;"),
    "nnf_ignored": ("if (op == O_NOT && (r->op_mask & O_NNF) && x != r->cost[O_ATOM]) continue;", ";"),
}
# the canonical order of Sec. 3: neighbouring connectives exchanged, splits taken with
# a descending, the pairs of a split column-major
_ORDER = "static const int order[7] = { O_F, O_U, O_G, O_X, O_AND, O_OR, O_NOT };"
_NAMES = ["O_F", "O_U", "O_G", "O_X", "O_AND", "O_OR", "O_NOT"]
for _k in range(6):
    _sw = list(_NAMES)
    _sw[_k], _sw[_k + 1] = _sw[_k + 1], _sw[_k]
    MUTANTS[f"order_swap_{_NAMES[_k][2:]}_{_NAMES[_k + 1][2:]}"] = (
        _ORDER, "static const int order[7] = { " + ", ".join(_sw) + " };")
_U_LOOP = """} else if (op == O_U) {
            for (int a = 1; a < x; ++a) {
                int b = x - a;
                if (!level_exists(r, a) || !level_exists(r, b)) continue;
                for (int64_t i = 0; i < r->L[a].n; ++i)
                    for (int64_t j = 0; j < r->L[b].n; ++j) batch_emit(B, op, a, i, b, j);"""
MUTANTS["splits_descending"] = (_U_LOOP, _U_LOOP.replace("for (int a = 1; a < x; ++a)",
                                                         "for (int a = x - 1; a >= 1; --a)"))
MUTANTS["pairs_column_major"] = (_U_LOOP, _U_LOOP.replace(
    """for (int64_t i = 0; i < r->L[a].n; ++i)
                    for (int64_t j = 0; j < r->L[b].n; ++j) batch_emit(B, op, a, i, b, j);""",
    """for (int64_t j = 0; j < r->L[b].n; ++j)
                    for (int64_t i = 0; i < r->L[a].n; ++i) batch_emit(B, op, a, i, b, j);"""))


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
                        "-k", "worked or bruteforce_levels or planted_tiny or identities or exhaustive or canonical_order_first"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

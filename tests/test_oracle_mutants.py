"""Planted mistakes in the oracle must each trip at least one pin (CPU only).

Each mutant is a copy of oracle_dgemm.c with one textual change -- a dropped
term, a wrong index, a transposed operand, a wrong sign, a missing scale or
check -- compiled with the oracle's own flags into a temporary directory and
loaded beside the real oracle. The pins in oracle_pins.py are then run against
it; the test fails if every pin still passes. Pins run in a child process,
because a mutant with a wrong index may write out of bounds: a crash counts as
caught, a clean pass of every pin as survived.
"""
import os
import shutil
import subprocess
import sys

import pytest

from oracle.build import HERE as ORACLE_DIR, build

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)

CHILD = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, oracle_pins
lib = oracle.load_library({so!r})
caught = []
for pin in oracle_pins.ALL_PINS:
    try:
        pin(lib)
    except AssertionError:
        caught.append(pin.__name__)
print("caught by:", caught)
sys.exit(1 if caught else 0)
"""

MUTANTS = {
    "dropped_last_term": ("for (int64_t p = 0; p < k; ++p)\n                s = s + op_a",
                          "for (int64_t p = 0; p < k - 1; ++p)\n                s = s + op_a"),
    "dropped_first_term": ("for (int64_t p = 0; p < k; ++p)\n                s = s + op_a",
                           "for (int64_t p = 1; p < k; ++p)\n                s = s + op_a"),
    "op_a_transposed": ("return ta ? A[i * lda + p] : A[p * lda + i];",
                        "return ta ? A[p * lda + i] : A[i * lda + p];"),
    "op_b_transposed": ("return tb ? B[p * ldb + j] : B[j * ldb + p];",
                        "return tb ? B[j * ldb + p] : B[p * ldb + j];"),
    "op_a_wrong_ld": ("return ta ? A[i * lda + p] : A[p * lda + i];",
                      "return ta ? A[i * lda + p] : A[p * lda + i + (lda > 1)];"),
    "beta_sign": ("*c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;",
                  "*c = (beta == 0.0) ? alpha * s : alpha * s - beta * *c;"),
    "alpha_dropped_beta0": ("*c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;",
                            "*c = (beta == 0.0) ? s : alpha * s + beta * *c;"),
    "beta0_reads_c": ("*c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;",
                      "*c = alpha * s + beta * *c;"),
    "c_index_swapped": ("double *c = &C[j * ldc + i];", "double *c = &C[i * ldc + j];"),
    "product_sign": ("s = s + op_a(ta, A, lda, i, p) * op_b(tb, B, ldb, p, j);",
                     "s = s - op_a(ta, A, lda, i, p) * op_b(tb, B, ldb, p, j);"),
    "k_zero_ignores_beta": ("C[j * ldc + i] = (beta == 0.0) ? 0.0 : beta * C[j * ldc + i];",
                            "C[j * ldc + i] = (beta == 0.0) ? 0.0 : C[j * ldc + i];"),
    "ldc_checked_against_n": ("if (ldc < max1(m)) return 13;", "if (ldc < max1(n)) return 13;"),
    "lda_unchecked_for_trans": ("int64_t rows_a = is_notrans(transa) ? m : k;",
                                "int64_t rows_a = m;"),
    "absden_missing_abs": ("s = s + fabs(op_a(ta, A, lda, i, p)) * fabs(op_b(tb, B, ldb, p, j));",
                           "s = s + op_a(ta, A, lda, i, p) * fabs(op_b(tb, B, ldb, p, j));"),
    "quick_return_any_beta": ("if (no_product && beta == 1.0) return 0;",
                              "if (no_product) return 0;"),
    "dd_product_error_dropped": ("*r = fma(a, b, -x);", "*r = 0.0 * fma(a, b, -x);"),
    "dd_sum_error_dropped": ("c = c + (q + r);", "c = c + r;"),
    "dd_twosum_sign": ("*e = (a - (x - z)) + (b - z);", "*e = (a - (x - z)) - (b - z);"),
    "dd_alpha_low_dropped": ("tr = tr + alpha * c;", "tr = alpha * c;"),
    "dd_beta_low_dropped": ("C[j * ldc + i] = v + (vr + (tr + ur));",
                            "C[j * ldc + i] = v + (vr + tr);"),
    "dd_op_b_first_only": ("two_prod(op_a(ta, A, lda, i, p), op_b(tb, B, ldb, p, j), &h, &r);",
                           "two_prod(op_a(ta, A, lda, i, p), op_b(tb, B, ldb, 0, j), &h, &r);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "oracle_dgemm.c")).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    d = tmp_path / "mut"
    d.mkdir()
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), d / "oracle.h")
    (d / "oracle_dgemm.c").write_text(src.replace(old, new))
    so = str(d / "liboracle_mut.so")
    build(out=so, sources=[str(d / "oracle_dgemm.c")])
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, tests=TESTS, so=so)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin\n{r.stdout}{r.stderr}"

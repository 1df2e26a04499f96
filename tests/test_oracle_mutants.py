"""Planted mistakes in the oracle must each trip at least one pin (CPU only).

Each mutant is a copy of the oracle's sources with one textual change in one
file -- a dropped term, a wrong index, a transposed operand, a wrong sign, a
missing scale or check -- compiled with the oracle's own flags into a temporary
directory and loaded beside the real oracle. The pins in oracle_pins.py and
blas3_pins.py are then run against
it; the test fails if every pin still passes. Pins run in a child process,
because a mutant with a wrong index may write out of bounds: a crash counts as
caught, a clean pass of every pin as survived.
"""
import os
import shutil
import subprocess
import sys

import pytest

from oracle.build import HERE as ORACLE_DIR, SOURCES, build

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)

CHILD = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, oracle_pins, blas3_pins
lib = oracle.load_library({so!r})
caught = []
for pin in oracle_pins.ALL_PINS + blas3_pins.ALL_PINS:
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


BLAS3_MUTANTS = {
    "syrk_same_row_twice": ("s = s + op_el(ta, A, lda, i, p) * op_el(ta, A, lda, j, p);",
                            "s = s + op_el(ta, A, lda, i, p) * op_el(ta, A, lda, i, p);"),
    "syrk_diagonal_skipped": ("int64_t i0 = lower ? j : 0, i1 = lower ? n - 1 : j;",
                              "int64_t i0 = lower ? j + 1 : 0, i1 = lower ? n - 1 : j;"),
    "syrk_whole_column": ("int64_t i0 = lower ? j : 0, i1 = lower ? n - 1 : j;",
                          "int64_t i0 = 0, i1 = n - 1;"),
    "syrk_beta_sign": ("*c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;",
                       "*c = (beta == 0.0) ? alpha * s : alpha * s - beta * *c;"),
    "syrk_lda_against_n": ("if (lda < max1(ta ? k : n)) return 7;", "if (lda < max1(n)) return 7;"),
    "tri_orientation_ignores_trans": ("int op_lower = is_lower(uplo) != ta;\n    double *W",
                                      "int op_lower = is_lower(uplo);\n    double *W"),
    "trmm_unit_reads_diagonal": ("return unit ? 1.0 : op_el(ta, A, lda, i, i);",
                                 "return op_el(ta, A, lda, i, i);"),
    "trmm_first_term_dropped": ("static int64_t tri_first(int op_lower, int64_t i) { return op_lower ? 0 : i; }",
                                "static int64_t tri_first(int op_lower, int64_t i) { return op_lower ? 1 : i; }"),
    "trmm_right_operands_swapped": ("s = s + B[p * ldb + i] * op_tri(ta, unit, A, lda, p, j);",
                                    "s = s + B[p * ldb + i] * op_tri(ta, unit, A, lda, j, p);"),
    "trmm_alpha_dropped": ("W[j * m + i] = alpha * s;", "W[j * m + i] = s;"),
    "trsm_left_wrong_order": ("int64_t i = op_lower ? t : m - 1 - t;", "int64_t i = t;"),
    "trsm_left_no_divide": ("x[i] = unit ? r : r / op_diag(ta, unit, A, lda, i);", "x[i] = r;"),
    "trsm_left_sum_sign": ("double r = alpha * x[i] - s;", "double r = alpha * x[i] + s;"),
    "trsm_right_transposed": ("s = s + B[p * ldb + i] * op_el(ta, A, lda, p, j);",
                              "s = s + B[p * ldb + i] * op_el(ta, A, lda, j, p);"),
    "trsm_right_alpha_dropped": ("double r = alpha * B[j * ldb + i] - s;", "double r = B[j * ldb + i] - s;"),
    "trsm_right_orientation": ("int op_lower = is_lower(uplo) != ta;\n\n    if (is_left(side))",
                               "int op_lower = is_lower(uplo);\n\n    if (is_left(side))"),
    "tri_lda_against_m": ("int64_t na = is_left(side) ? m : n; /* order of A */",
                          "int64_t na = m; /* order of A */"),
    "tri_alpha0_keeps_b": ("for (int64_t i = 0; i < m; ++i) B[j * ldb + i] = 0.0;\n        return 0;\n    }\n    int ta = is_trans(transa), unit = is_unit(diag), left",
                           "for (int64_t i = 0; i < m; ++i) B[j * ldb + i] = B[j * ldb + i];\n        return 0;\n    }\n    int ta = is_trans(transa), unit = is_unit(diag), left"),
}

CASES = [("oracle_dgemm.c", k, *v) for k, v in MUTANTS.items()] + \
        [("oracle_blas3.c", k, *v) for k, v in BLAS3_MUTANTS.items()]


@pytest.mark.parametrize("fname,name,old,new", CASES, ids=[c[1] for c in CASES])
def test_mutant_is_caught(fname, name, old, new, tmp_path):
    src = open(os.path.join(ORACLE_DIR, fname)).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    d = tmp_path / "mut"
    d.mkdir()
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), d / "oracle.h")
    for path in SOURCES:
        shutil.copy(path, d / os.path.basename(path))
    (d / fname).write_text(src.replace(old, new))
    so = str(d / "liboracle_mut.so")
    build(out=so, sources=[str(d / os.path.basename(path)) for path in SOURCES])
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, tests=TESTS, so=so)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin\n{r.stdout}{r.stderr}"

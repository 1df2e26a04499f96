/*
 * oracle_blas3.c -- plain CPU evaluation of three level-3 BLAS operations that
 * can be cast in terms of GEMM: the symmetric rank-k update (dsyrk), the
 * triangular matrix-matrix multiply (dtrmm) and the triangular solve with many
 * right-hand sides (dtrsm).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, never by the product
 * library. Built with the same flags as oracle_dgemm.c (no FMA contraction, no
 * fast math), so every product and every sum is one rounded binary64 operation.
 *
 * The paper's Step 2 ("Poorman's BLAS") names these operations: the level-3
 * BLAS that a tuned GEMM lets one build (Kagstrom, Ling and Van Loan, 1998).
 * Their definitions, argument lists and argument checks are those of the
 * level-3 BLAS (Dongarra, Du Croz, Hammarling and Duff, 1990), cited by the
 * paper's section 1.1; storage is column-major with leading dimensions
 * (section 2.3). Nothing here is blocked: every entry is its definition written
 * out, with sums over p taken in increasing order from zero and the scalar
 * factors applied afterwards, and the triangular solve is plain substitution.
 * Only the triangle of A (or C) that `uplo` names is read or written; with a
 * unit diagonal the stored diagonal of A is not read.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

static int is_notrans(char t) { return t == 'N' || t == 'n'; }
static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static int is_lower(char u) { return u == 'L' || u == 'l'; }
static int is_upper(char u) { return u == 'U' || u == 'u'; }
static int is_left(char s) { return s == 'L' || s == 'l'; }
static int is_right(char s) { return s == 'R' || s == 'r'; }
static int is_unit(char d) { return d == 'U' || d == 'u'; }
static int is_nonunit(char d) { return d == 'N' || d == 'n'; }
static int64_t max1(int64_t x) { return x > 1 ? x : 1; }

/* op(A)(i, p) for a stored A: A itself (ta = 0) or its transpose (ta = 1). */
static double op_el(int ta, const double *A, int64_t lda, int64_t i, int64_t p)
{
    return ta ? A[i * lda + p] : A[p * lda + i];
}

/*
 * Triangular op(A): it is lower triangular when A is lower and not transposed
 * or upper and transposed. tri_first/tri_last give the range of p for which
 * op(A)(i, p) lies in the triangle (row i); the diagonal is 1 when unit.
 */
static int64_t tri_first(int op_lower, int64_t i) { return op_lower ? 0 : i; }
static int64_t tri_last(int op_lower, int64_t i, int64_t na) { return op_lower ? i : na - 1; }

static double op_diag(int ta, int unit, const double *A, int64_t lda, int64_t i)
{
    return unit ? 1.0 : op_el(ta, A, lda, i, i);
}

/* op(A)(i, p) inside the triangle, the diagonal taken as 1 when unit. */
static double op_tri(int ta, int unit, const double *A, int64_t lda, int64_t i, int64_t p)
{
    return i == p ? op_diag(ta, unit, A, lda, i) : op_el(ta, A, lda, i, p);
}

/*
 * C := alpha*op(A)*op(A)^T + beta*C on the `uplo` triangle of the n-by-n C;
 * op(A) is n-by-k: A (trans 'N', stored n-by-k) or A^T (trans 'T', stored
 * k-by-n). The other triangle of C is neither read nor written.
 * Returns 0 or the 1-based position of the first bad argument.
 */
int oracle_dsyrk(char uplo, char trans, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, double beta, double *C, int64_t ldc)
{
    if (!is_lower(uplo) && !is_upper(uplo)) return 1;
    if (!is_notrans(trans) && !is_trans(trans)) return 2;
    if (n < 0) return 3;
    if (k < 0) return 4;
    int ta = is_trans(trans);
    int no_product = (alpha == 0.0 || k == 0);
    if (n > 0 && !no_product && A == NULL) return 6;
    if (lda < max1(ta ? k : n)) return 7;
    if (n > 0 && C == NULL) return 9;
    if (ldc < max1(n)) return 10;
    if (n == 0) return 0;
    if (no_product && beta == 1.0) return 0;

    int lower = is_lower(uplo);
    int nt = oracle_get_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        int64_t i0 = lower ? j : 0, i1 = lower ? n - 1 : j; /* rows of column j in the triangle */
        for (int64_t i = i0; i <= i1; ++i) {
            double *c = &C[j * ldc + i];
            if (no_product) {
                *c = (beta == 0.0) ? 0.0 : beta * *c;
                continue;
            }
            double s = 0.0;
            for (int64_t p = 0; p < k; ++p)
                s = s + op_el(ta, A, lda, i, p) * op_el(ta, A, lda, j, p);
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;
        }
    }
    return 0;
}

/* Checks shared by dtrmm and dtrsm, in their argument order. */
static int check_tri(char side, char uplo, char transa, char diag, int64_t m, int64_t n,
                     const double *A, int64_t lda, const double *B, int64_t ldb,
                     int needs_a)
{
    if (!is_left(side) && !is_right(side)) return 1;
    if (!is_lower(uplo) && !is_upper(uplo)) return 2;
    if (!is_notrans(transa) && !is_trans(transa)) return 3;
    if (!is_unit(diag) && !is_nonunit(diag)) return 4;
    if (m < 0) return 5;
    if (n < 0) return 6;
    int64_t na = is_left(side) ? m : n; /* order of A */
    if (needs_a && m > 0 && n > 0 && A == NULL) return 8;
    if (lda < max1(na)) return 9;
    if (m > 0 && n > 0 && B == NULL) return 10;
    if (ldb < max1(m)) return 11;
    return 0;
}

/*
 * B := alpha*op(A)*B (side 'L', A m-by-m) or B := alpha*B*op(A) (side 'R',
 * A n-by-n); B is m-by-n and is overwritten. alpha == 0 sets B to zero without
 * reading A or B. Returns 0, the position of the first bad argument, or -1 if
 * the temporary result cannot be allocated.
 */
int oracle_dtrmm(char side, char uplo, char transa, char diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    int info = check_tri(side, uplo, transa, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (info) return info;
    if (m == 0 || n == 0) return 0;
    int nt = oracle_get_threads();
    if (alpha == 0.0) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) B[j * ldb + i] = 0.0;
        return 0;
    }
    int ta = is_trans(transa), unit = is_unit(diag), left = is_left(side);
    int op_lower = is_lower(uplo) != ta;
    double *W = malloc((size_t)(m * n) * sizeof(double)); /* result, m-by-n, ld m */
    if (W == NULL) return -1;

#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (left) { /* sum over p of op(A)(i, p) B(p, j), p in row i's triangle */
                for (int64_t p = tri_first(op_lower, i); p <= tri_last(op_lower, i, m); ++p)
                    s = s + op_tri(ta, unit, A, lda, i, p) * B[j * ldb + p];
            } else {    /* sum over p of B(i, p) op(A)(p, j), p in column j's triangle */
                int64_t p0 = op_lower ? j : 0, p1 = op_lower ? n - 1 : j;
                for (int64_t p = p0; p <= p1; ++p)
                    s = s + B[p * ldb + i] * op_tri(ta, unit, A, lda, p, j);
            }
            W[j * m + i] = alpha * s;
        }
    }
    for (int64_t j = 0; j < n; ++j) memcpy(&B[j * ldb], &W[j * m], (size_t)m * sizeof(double));
    free(W);
    return 0;
}

/*
 * Solves op(A)*X = alpha*B (side 'L', A m-by-m) or X*op(A) = alpha*B (side
 * 'R', A n-by-n) for the m-by-n X, which overwrites B. Substitution: for side
 * 'L' each column of B is solved on its own, for side 'R' each row; entries are
 * found in the order in which the triangle makes them available (forward for
 * a lower op(A) on the left, backward for an upper one; the reverse on the
 * right). There is no test for singularity: a zero diagonal divides by zero.
 * alpha == 0 sets B to zero without reading A or B.
 */
int oracle_dtrsm(char side, char uplo, char transa, char diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    int info = check_tri(side, uplo, transa, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (info) return info;
    if (m == 0 || n == 0) return 0;
    int nt = oracle_get_threads();
    if (alpha == 0.0) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) B[j * ldb + i] = 0.0;
        return 0;
    }
    int ta = is_trans(transa), unit = is_unit(diag);
    int op_lower = is_lower(uplo) != ta;

    if (is_left(side)) {
        /* Column j: op(A)(i, i) x_i = alpha b_i - sum over p != i in row i's triangle of
           op(A)(i, p) x_p. */
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            double *x = &B[j * ldb];
            for (int64_t t = 0; t < m; ++t) {
                int64_t i = op_lower ? t : m - 1 - t;
                double s = 0.0;
                int64_t p0 = op_lower ? 0 : i + 1, p1 = op_lower ? i - 1 : m - 1;
                for (int64_t p = p0; p <= p1; ++p) s = s + op_el(ta, A, lda, i, p) * x[p];
                double r = alpha * x[i] - s;
                x[i] = unit ? r : r / op_diag(ta, unit, A, lda, i);
            }
        }
    } else {
        /* Row i: x_j op(A)(j, j) = alpha b_j - sum over p != j in column j's triangle of
           x_p op(A)(p, j). */
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t t = 0; t < n; ++t) {
                int64_t j = op_lower ? n - 1 - t : t;
                double s = 0.0;
                int64_t p0 = op_lower ? j + 1 : 0, p1 = op_lower ? n - 1 : j - 1;
                for (int64_t p = p0; p <= p1; ++p) s = s + B[p * ldb + i] * op_el(ta, A, lda, p, j);
                double r = alpha * B[j * ldb + i] - s;
                B[j * ldb + i] = unit ? r : r / op_diag(ta, unit, A, lda, j);
            }
        }
    }
    return 0;
}

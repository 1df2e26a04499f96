/*
 * oracle_dgemm.c -- plain CPU evaluation of double-precision GEMM.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * Built with gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp: every product
 * and every sum is a separately rounded binary64 operation (round to nearest
 * even, no fused multiply-add, no flush of subnormals).
 *
 * The computation is the definition in the paper's notation (section 1.2 for the
 * four transpose cases and alpha/beta; section 2.1 for the entrywise sum and its
 * loop over i, j, p; section 2.3 for column-major storage with leading
 * dimensions). Each entry c_ij is accumulated over p = 0, 1, ..., k-1 in that
 * order, starting from zero; then alpha and beta are applied. The loop over
 * columns j is split over OpenMP threads; since no entry is shared between
 * threads, the result is bitwise the same for every thread count.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <omp.h>

static int g_threads = 0; /* 0: OpenMP default */

void oracle_set_threads(int nthreads) { g_threads = nthreads > 0 ? nthreads : 0; }

int oracle_get_threads(void) { return g_threads > 0 ? g_threads : omp_get_max_threads(); }

static int is_notrans(char t) { return t == 'N' || t == 'n'; }
static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static int64_t max1(int64_t x) { return x > 1 ? x : 1; }

/* op(A)(i,p): A is m-by-k stored as is, or k-by-m stored and transposed. */
static double op_a(int ta, const double *A, int64_t lda, int64_t i, int64_t p)
{
    return ta ? A[i * lda + p] : A[p * lda + i];
}

/* op(B)(p,j): B is k-by-n stored as is, or n-by-k stored and transposed. */
static double op_b(int tb, const double *B, int64_t ldb, int64_t p, int64_t j)
{
    return tb ? B[p * ldb + j] : B[j * ldb + p];
}

/*
 * Argument checks in the order the arguments appear in the dgemm call. Returns
 * 0 or the 1-based position of the first bad argument. `needs_ab` says whether
 * A and B will be dereferenced, `needs_c` whether C will be.
 */
static int check_args(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      const double *A, int64_t lda, const double *B, int64_t ldb,
                      const double *C, int64_t ldc, int needs_ab, int needs_c)
{
    if (!is_notrans(transa) && !is_trans(transa)) return 1;
    if (!is_notrans(transb) && !is_trans(transb)) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    int64_t rows_a = is_notrans(transa) ? m : k; /* rows of the stored A */
    int64_t rows_b = is_notrans(transb) ? k : n; /* rows of the stored B */
    if (needs_ab && A == NULL) return 7;
    if (lda < max1(rows_a)) return 8;
    if (needs_ab && B == NULL) return 9;
    if (ldb < max1(rows_b)) return 10;
    if (needs_c && C == NULL) return 12;
    if (ldc < max1(m)) return 13;
    return 0;
}

int oracle_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc)
{
    int empty = (m == 0 || n == 0);
    int no_product = (alpha == 0.0 || k == 0);
    int info = check_args(transa, transb, m, n, k, A, lda, B, ldb, C, ldc,
                          !empty && !no_product, !empty);
    if (info) return info;
    if (empty) return 0;
    if (no_product && beta == 1.0) return 0;

    int ta = is_trans(transa), tb = is_trans(transb);
    int nt = oracle_get_threads();

    if (no_product) {
        /* C := beta*C; with beta == 0 the old C is not read. */
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i)
                C[j * ldc + i] = (beta == 0.0) ? 0.0 : beta * C[j * ldc + i];
        return 0;
    }

#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t p = 0; p < k; ++p)
                s = s + op_a(ta, A, lda, i, p) * op_b(tb, B, ldb, p, j);
            double *c = &C[j * ldc + i];
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;
        }
    }
    return 0;
}

int oracle_dgemm_absden(char transa, char transb, int64_t m, int64_t n, int64_t k,
                        double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb,
                        double beta, const double *C0, int64_t ldc,
                        double *D, int64_t ldd)
{
    int empty = (m == 0 || n == 0);
    int no_product = (alpha == 0.0 || k == 0);
    int info = check_args(transa, transb, m, n, k, A, lda, B, ldb, C0, ldc,
                          !empty && !no_product, !empty && beta != 0.0);
    if (info) return info;
    if (!empty && D == NULL) return 14;
    if (ldd < max1(m)) return 15;
    if (empty) return 0;

    int ta = is_trans(transa), tb = is_trans(transb);
    int nt = oracle_get_threads();
    double aa = fabs(alpha), ab = fabs(beta);

#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (!no_product)
                for (int64_t p = 0; p < k; ++p)
                    s = s + fabs(op_a(ta, A, lda, i, p)) * fabs(op_b(tb, B, ldb, p, j));
            double d = aa * s;
            if (beta != 0.0) d = d + ab * fabs(C0[j * ldc + i]);
            D[j * ldd + i] = d;
        }
    }
    return 0;
}

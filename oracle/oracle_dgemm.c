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

/*
 * Extended-precision reference (not the parity target; it states the true error of
 * the oracle above, of the native kernel and of the split path). Each entry is the
 * same dot product evaluated with error-free transformations: the product of two
 * doubles is h + r exactly (TwoProduct: h = fl(a*b), r = fma(a, b, -h)), the sum of
 * two doubles is s + q exactly (TwoSum, Knuth), and the rounding errors r and q are
 * summed on the side (Ogita, Rump and Oishi, "Accurate sum and dot product", SIAM J.
 * Sci. Comput. 26(6), 2005, algorithm Dot2). The result is as accurate as a dot
 * product computed in twice the working precision and then rounded:
 * |s + c - x'y| <= u|x'y| + gamma_k^2 |x|'|y|. alpha and beta are applied to the
 * pair (s, c) with the same transformations before the single final rounding.
 */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *h, double *r)
{
    double x = a * b;
    *r = fma(a, b, -x);
    *h = x;
}

int oracle_dgemm_dd(char transa, char transb, int64_t m, int64_t n, int64_t k,
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
    if (beta == 1.0 && no_product) return 0;

    int ta = is_trans(transa), tb = is_trans(transb);
    int nt = oracle_get_threads();

#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0, c = 0.0;
            if (!no_product) {
                for (int64_t p = 0; p < k; ++p) {
                    double h, r, q;
                    two_prod(op_a(ta, A, lda, i, p), op_b(tb, B, ldb, p, j), &h, &r);
                    two_sum(s, h, &s, &q);
                    c = c + (q + r);
                }
            }
            /* alpha*(s + c) + beta*c0, rounded once at the end */
            double t, tr, u = 0.0, ur = 0.0, v, vr;
            two_prod(alpha, s, &t, &tr);
            tr = tr + alpha * c;
            if (beta != 0.0) two_prod(beta, C[j * ldc + i], &u, &ur);
            two_sum(t, u, &v, &vr);
            C[j * ldc + i] = v + (vr + (tr + ur));
        }
    }
    return 0;
}

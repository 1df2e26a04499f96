/*
 * oracle.h -- plain CPU evaluation of double-precision GEMM.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library includes, links or
 * calls this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do. It shares no header, helper or constant with the HIP path.
 *
 * What it computes (paper, section 1.2, the dgemm statement of the problem):
 *
 *     C := alpha * op(A) * op(B) + beta * C,    op(X) = X or X^T,
 *
 * with C m-by-n, op(A) m-by-k, op(B) k-by-n, all stored column-major with a
 * leading dimension (paper, section 2.3: element (i,j) of C lives at
 * C[j*ldc + i]). Each entry is the dot product of section 2.1,
 * c_ij = sum_{p=0}^{k-1} a_ip b_pj, accumulated in ascending p, every product
 * and every sum rounded to binary64 (the library is built without FMA
 * contraction), then combined with the old C as alpha*s + beta*c.
 *
 * Readings where the paper is silent (BLAS conventions the paper invokes):
 *   - trans characters: 'N'/'n' means op(X) = X; 'T'/'t'/'C'/'c' mean
 *     op(X) = X^T (real data, so conjugate transpose is transpose);
 *   - beta == 0 means the old C is never read (it may hold NaN);
 *   - alpha == 0 or k == 0 means A and B are never read: C := beta*C;
 *   - return 0 on success, else the 1-based position of the first invalid
 *     argument in the argument list (1 transa, 2 transb, 3 m, 4 n, 5 k,
 *     7 A, 8 lda, 9 B, 10 ldb, 12 C, 13 ldc). A null pointer is an error only
 *     where it would be dereferenced. On error nothing is written.
 */
#ifndef ORACLE_DGEMM_H
#define ORACLE_DGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The definition itself, evaluated in place on host memory. */
int oracle_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc);

/*
 * Companion error denominator: D(i,j) = |alpha| * sum_p |op(A)(i,p)| |op(B)(p,j)|
 * + |beta| * |C0(i,j)|, written to D (column-major, leading dimension ldd);
 * C0 is read only when beta != 0. Same argument checks as oracle_dgemm, plus
 * 14 for a null D and 15 for ldd < max(1, m).
 */
int oracle_dgemm_absden(char transa, char transb, int64_t m, int64_t n, int64_t k,
                        double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb,
                        double beta, const double *C0, int64_t ldc,
                        double *D, int64_t ldd);

/*
 * The same operation with each entry evaluated in doubled working precision
 * (error-free TwoProduct and TwoSum with the errors summed on the side, the Dot2
 * algorithm of Ogita, Rump and Oishi, 2005) and rounded once at the end: within
 * about one rounding of the exact result, so it states the true error of the
 * routine above and of the GPU paths. Same arguments, checks and conventions as
 * oracle_dgemm. Not a parity target.
 */
int oracle_dgemm_dd(char transa, char transb, int64_t m, int64_t n, int64_t k,
                    double alpha, const double *A, int64_t lda,
                    const double *B, int64_t ldb,
                    double beta, double *C, int64_t ldc);

/* Level-3 BLAS built on the same definitions (oracle_blas3.c): symmetric rank-k
   update, triangular multiply, triangular solve. Arguments in level-3 BLAS order;
   each returns 0 or the 1-based position of the first bad argument (dtrmm: -1 if
   its temporary cannot be allocated). */
int oracle_dsyrk(char uplo, char trans, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, double beta, double *C, int64_t ldc);
int oracle_dtrmm(char side, char uplo, char transa, char diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb);
int oracle_dtrsm(char side, char uplo, char transa, char diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb);

/* Number of OpenMP threads the routines above use (<= 0 resets to the default). */
void oracle_set_threads(int nthreads);
int oracle_get_threads(void);

#ifdef __cplusplus
}
#endif

#endif

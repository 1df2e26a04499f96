/*
 * mdg.h -- double-precision GEMM for AMD Instinct MI355X (gfx950), C ABI.
 *
 * The operation is the BLAS dgemm the paper states in section 1.2:
 *
 *     C := alpha * op(A) * op(B) + beta * C,     op(X) = X or X^T,
 *
 * where C is m x n, op(A) is m x k and op(B) is k x n ("k is the third
 * dimension"). Every matrix is stored column-major inside a larger array with a
 * leading dimension (paper, section 2.3: element (i,j) of C is C[j*ldc + i]).
 *
 * Arguments (all entry points below that take them):
 *   transa, transb  'N' or 'n': op(X) = X.  'T', 't', 'C' or 'c': op(X) = X^T
 *                   (the data are real, so conjugate transpose is transpose).
 *   m, n, k         sizes, >= 0.
 *   alpha, beta     scalars, passed by value.
 *   A, lda          device pointer to A; stored A is m x k when transa is N,
 *                   k x m when it is T; lda >= max(1, rows of stored A).
 *   B, ldb          device pointer to B; stored B is k x n (N) or n x k (T);
 *                   ldb >= max(1, rows of stored B).
 *   C, ldc          device pointer to C (m x n), ldc >= max(1, m). Rows m..ldc-1
 *                   of each column are never read or written.
 *   stream          a hipStream_t (NULL = the null stream). Work is enqueued on
 *                   it asynchronously; the call does not wait for completion.
 *
 * Ownership: A, B and C belong to the caller, who keeps them alive and does not
 * modify A, B or C until the enqueued work has completed on `stream`. The
 * library never allocates, frees or retains them, and the entry points in this
 * header use no workspace. C must not overlap A or B (not checked).
 *
 * Conventions (BLAS, as the paper's dgemm call implies):
 *   - beta == 0: C is not read on entry (it may hold NaN or garbage).
 *   - alpha == 0 or k == 0: A and B are not read (may be NULL); C := beta*C.
 *   - m == 0 or n == 0, or (alpha == 0 or k == 0) and beta == 1: nothing is
 *     enqueued and no pointer is dereferenced.
 *
 * Return value: MDG_SUCCESS (0); a positive value is the 1-based position of
 * the first invalid argument in the dgemm argument list, in the order the
 * reference BLAS checks them (1 transa, 2 transb, 3 m < 0, 4 n < 0, 5 k < 0,
 * 7 A == NULL where it would be read, 8 lda too small, 9 B == NULL, 10 ldb too
 * small, 12 C == NULL where it would be touched, 13 ldc too small); a negative
 * value is a runtime error (MDG_ERR_*). On any error nothing is enqueued and C
 * is untouched. No entry point prints or aborts.
 *
 * Thread safety: every entry point is reentrant; the only global state is a
 * read-only table of kernel variants and a per-device memo of the architecture
 * check.
 */
#ifndef MDG_H
#define MDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDG_SUCCESS 0
#define MDG_ERR_HIP (-1)     /* a HIP call failed (no device, launch error) */
#define MDG_ERR_VARIANT (-2) /* unknown kernel variant id, or one unfit for the arguments */
#define MDG_ERR_DEVICE (-3)  /* the current device is not gfx950 */
#define MDG_ERR_SIZE (-4)    /* m, n too large for one launch's grid */

#define MDG_VARIANT_AUTO (-1)

/*
 * C := alpha*op(A)*op(B) + beta*C on the current HIP device, enqueued on
 * `stream`. The kernel variant is chosen from the shape (see
 * mdg_select_variant).
 */
int mdg_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
              double alpha, const double *A, int64_t lda,
              const double *B, int64_t ldb,
              double beta, double *C, int64_t ldc, void *stream);

/*
 * The same operation with an explicit kernel variant (0 .. mdg_num_variants()-1,
 * or MDG_VARIANT_AUTO). Every variant computes the same result to rounding;
 * integer-valued inputs give bitwise-identical results in every variant.
 * Returns MDG_ERR_VARIANT for an unknown id.
 */
int mdg_dgemm_ex(int variant, char transa, char transb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc, void *stream);

/*
 * The variant mdg_dgemm would launch for these arguments, or -1 when it would
 * launch no GEMM kernel (quick return, or the alpha == 0 / k == 0 scaling
 * path). Pure host function: no HIP call, no pointer dereference.
 */
int mdg_select_variant(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       double alpha, double beta);

/* Number of kernel variants, and a static name for each (NULL if out of range). */
int mdg_num_variants(void);
const char *mdg_variant_name(int variant);

/*
 * Geometry of a variant: macro-tile rows (mt), columns (nt), k-panel depth (kt)
 * and threads per workgroup. Returns 0, or MDG_ERR_VARIANT.
 */
int mdg_variant_info(int variant, int *mt, int *nt, int *kt, int *threads);

/* Static description of a status code (never NULL). */
const char *mdg_status_string(int status);

/*
 * The raw hipError_t of the last HIP call that failed inside this library on the
 * calling thread (0 if none): the detail behind an MDG_ERR_HIP return.
 */
int mdg_last_hip_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int mdg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDG_H */

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
#define MDG_ERR_SIZE (-4)    /* m, n too large for one launch's grid, or a leading dimension so
                                large that the part of one k-panel inside the matrix spans 4 GiB
                                or more (the kernels address it by 32-bit byte offsets) */
#define MDG_ERR_SCRATCH (-5) /* the problem needs more scratch than the no-allocation entry point
                                holds (mdg_dgemm_split_noalloc_max_bytes) */

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
 * The tiled variant mdg_dgemm would launch for these arguments, or -1 when it
 * would launch none (quick return, the alpha == 0 / k == 0 scaling path, or a
 * C with at most 16 rows or columns computed by the thin kernel alone). The
 * variant may cover only the leading block of C: see mdg_dgemm_plan. Pure
 * host function: no HIP call, no pointer dereference.
 */
int mdg_select_variant(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       double alpha, double beta);

/*
 * How mdg_dgemm (automatic variant) splits a product with m, n, k >= 1 (paper,
 * section 2.4: the fringes left when m, n are not multiples of the block
 * sizes). *variant (or -1: none) computes rows [0, *m_main) and columns
 * [0, *n_main) of C with its tiles; one launch of the thin kernel computes the
 * rest, rows [*m_main, m) over all columns and columns [*n_main, n) over rows
 * [0, *m_main), each at most 16 wide. A C with at most 16 rows or columns may
 * be computed by the thin kernel alone (*variant = -1, *m_main = *n_main = 0).
 * Returns 0, or the 1-based position of the first invalid argument (bad
 * transpose letter, m, n or k below 1, or a NULL output pointer). Pure host
 * function: no HIP call.
 */
int mdg_dgemm_plan(char transa, char transb, int64_t m, int64_t n, int64_t k, int *variant,
                   int64_t *m_main, int64_t *n_main);

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

/* ------------------------------------------------------------------------------------------
 * Split-precision FP64 GEMM on the INT8 matrix cores (Ozaki scheme; not in the paper, which
 * computes dgemm in FP64 only -- this is the same operation of section 1.2, emulated).
 *
 * op(A) is scaled row by row and op(B) column by column by powers of two so every entry lies in
 * (-1, 1), each scaled entry is split exactly into `nslices` int8 slices of 7 bits, the products
 * of slice pairs (s, t) with s + t <= nslices + 1 are formed exactly in INT32 on the INT8
 * matrix cores (v_mfma_i32_32x32x32_i8 up to 8 slices, v_mfma_i32_16x16x64_i8 beyond), and the
 * sum is recombined, unscaled and combined with alpha, beta and the old C in binary64. The result approximates the FP64 product: the error is about
 * k * 2^(-7*nslices) times the product of the row and column maxima, so entries whose magnitudes
 * spread widely within a row or column need more slices. Measured for entries u * 2^e, e uniform in
 * [-phi, phi]: at k = 8192, nslices = 7 (phi = 0), 8 (phi = 8), 10 (phi = 32) keep
 * max |C - Cref| / (|A||B|)_ij below 1e-13; at k as small as 32, phi = 8 needs 9, and phi = 32 is
 * not reached even with 12 (a short row spanning 2^64 leaves (|A||B|)_ij far below the product of
 * the maxima). Non-finite inputs: a row of op(A) (column of op(B)) holding NaN or Inf makes that
 * whole row (column) of C NaN -- where IEEE arithmetic would give NaN or +-Inf there, the split
 * path gives NaN; NaN in the old C propagates through beta*C as usual.
 * ------------------------------------------------------------------------------------------ */

/* Largest supported `nslices` (the smallest is 1). */
int mdg_split_max_slices(void);

/*
 * Bytes of device workspace mdg_dgemm_split needs for these sizes, or -1 for invalid sizes or
 * slice count. Layout: the int8 slices of op(A) (rows = m) and of op(B)^T (rows = n), each in
 * the k-panel tiles described at mdg_split_slices, then int32 exponents of the m rows and n
 * columns, each part aligned to 256 bytes.
 */
int64_t mdg_dgemm_split_workspace_size(int64_t m, int64_t n, int64_t k, int nslices);

/*
 * C := alpha*op(A)*op(B) + beta*C by the split-precision scheme above. Arguments 1-13 and the
 * stream are as for mdg_dgemm; `workspace` is a caller-owned device buffer of at least
 * mdg_dgemm_split_workspace_size(m, n, k, nslices) bytes, 256-byte aligned, which the call
 * overwrites (it must stay untouched until the work completes on `stream`). Extra status codes:
 * 14 nslices out of range, 15 workspace NULL, too small or misaligned; MDG_ERR_SIZE when a slice
 * array exceeds 4 GiB. Conventions for m, n, k, alpha, beta zero are those of mdg_dgemm.
 */
int mdg_dgemm_split(char transa, char transb, int64_t m, int64_t n, int64_t k,
                    double alpha, const double *A, int64_t lda,
                    const double *B, int64_t ldb,
                    double beta, double *C, int64_t ldc,
                    int nslices, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * The slicing step alone, for one operand: operand 0 slices the rows of op(A) (rows = m, trans =
 * transa, X = A, ld = lda), operand 1 the columns of op(B) (rows = n, trans = transb, X = B,
 * ld = ldb). With rp = rows rounded up to a multiple of 128 and kp = k rounded up to a multiple
 * of 64, writes slice s of entry (r, p) at
 *   slices[s*rp*kp + (p/32)*rp*32 + (r/32)*1024 + 16*slot(r%32, (p/16)%2) + p%16],
 *   slot(i, h) = 2*i + (h XOR (((i/4) XOR (i/8)) AND 1)),
 * for r < rp, p < kp (zero for r >= rows or p >= k): each 32-deep k-panel of a slice is rp*32
 * bytes, made of 1 KiB chunks of 32 rows in which row i keeps its two 16-byte halves at slots
 * slot(i, 0) and slot(i, 1). `slices` holds nslices*rp*kp bytes; and exponents[r] = e with
 * max_p |x(r,p)| = f * 2^e, f in [0.5, 1) (0 for a zero row; 0x7FFFFFFF for a row holding NaN or
 * Inf, whose slices are then unspecified). Returns 0, or
 * 1 operand, 2 trans, 3 rows < 0, 4 k < 0, 5 X NULL, 6 ld too small, 7 nslices out of range,
 * 8 output NULL, or a negative runtime code.
 */
int mdg_split_slices(int operand, char trans, int64_t rows, int64_t k, const double *X, int64_t ld,
                     int nslices, int8_t *slices, int32_t *exponents, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mdg_dgemm_split without a workspace argument. The
 * slices and exponents go to a static device array of the library, mdg_dgemm_split_noalloc_max_bytes()
 * bytes (64 MiB) per GPU, allocated with the library's code on each device and held until the
 * process ends; the call itself allocates and frees nothing. Arguments 1-14, the stream, the
 * status codes and the result (bit for bit) are those of mdg_dgemm_split with a workspace of
 * mdg_dgemm_split_workspace_size(m, n, k, nslices) bytes; a problem whose workspace size exceeds
 * the array returns MDG_ERR_SCRATCH before any HIP call (for example m = n = k = 2048 fits with
 * up to 7 slices). Every call on one GPU shares that GPU's array: calls whose work overlaps on the
 * device (different streams, or host threads without ordering) race and give undefined results;
 * calls in order on one stream are safe. The exponent arrays are cleared by a kernel on `stream`
 * at the start of every call.
 */
int64_t mdg_dgemm_split_noalloc_max_bytes(void);

int mdg_dgemm_split_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k,
                            double alpha, const double *A, int64_t lda,
                            const double *B, int64_t ldb,
                            double beta, double *C, int64_t ldc,
                            int nslices, void *stream);

/* ------------------------------------------------------------------------------------------
 * Split-precision FP64 GEMM by the Chinese remainder theorem (Ozaki scheme II: Ozaki, Uchino and
 * Imamura 2025; the same operation of section 1.2, emulated).
 *
 * op(A) is scaled row by row and op(B) column by column to integers of w bits
 * (A'(i,p) = trunc(A(i,p) 2^(w - e_i)), e_i the binary exponent of the row maximum). For each of
 * `nmoduli` pairwise coprime moduli m_l (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211,
 * 199, 197, 193, 191, 181, 179, 173, 167, 163, 157, 151, 149, in this order) the symmetric int8
 * residues of A' and B' are multiplied exactly in INT32 on the INT8 matrix cores
 * (v_mfma_i32_32x32x32_i8) and reduced modulo m_l; the Chinese remainder theorem turns the residues
 * into the integer (A'B')(i,j) exactly, since w is the largest width (at most 72) with
 * 4 k 2^(2w) <= M = prod m_l; that integer is rounded once to binary64, unscaled, and combined with
 * alpha, beta and the old C in binary64. One INT8 product per modulus, against s(s+1)/2 slice
 * products for mdg_dgemm_split. The error comes from the w-bit scaling alone: measured on
 * u * 2^e data with e uniform in [-phi, phi], nmoduli = 14 (phi = 0), 15 (phi = 8), 16 (phi = 32)
 * keep max |C - Cref| / (|A||B|)_ij below 1e-13 at k = 2048 to 8192; at k = 32, phi = 8 needs 16.
 * Non-finite inputs: as mdg_dgemm_split (a row of op(A) or column of op(B) holding NaN or Inf makes
 * that row or column of C NaN).
 * ------------------------------------------------------------------------------------------ */

/* Largest supported `nmoduli` (the smallest is 1). */
int mdg_crt_max_moduli(void);

/* The width w (bits) the CRT path scales op(A) and op(B) to for this k and modulus count, or 0
 * if nmoduli is out of range (or too small for any width). Host only. */
int mdg_crt_bits(int64_t k, int nmoduli);

/*
 * Bytes of device workspace mdg_dgemm_crt needs, or -1 for invalid sizes or modulus count.
 * Layout (each part aligned to 256 bytes): the int8 residues of op(A) (rows = m) and op(B)^T
 * (rows = n) in the k-panel layout of mdg_split_slices (slice l = modulus l), the product residues
 * (nmoduli x m x ceil(n/4) 32-bit words: word (j/4)*m + i of modulus l holds the residues of
 * C(i, 4(j/4) .. 4(j/4)+3), one byte each), then int32 exponents of the m rows and n columns.
 */
int64_t mdg_dgemm_crt_workspace_size(int64_t m, int64_t n, int64_t k, int nmoduli);

/*
 * C := alpha*op(A)*op(B) + beta*C by the CRT scheme above. Arguments 1-13 and the stream are as
 * for mdg_dgemm; `workspace` is a caller-owned device buffer of at least
 * mdg_dgemm_crt_workspace_size(m, n, k, nmoduli) bytes, 256-byte aligned, which the call
 * overwrites. Extra status codes: 14 nmoduli out of range (or too few for this k), 15 workspace
 * NULL, too small or misaligned; MDG_ERR_SIZE when one modulus' residues of an operand exceed
 * 4 GiB. Conventions for m, n, k, alpha, beta zero are those of mdg_dgemm.
 */
int mdg_dgemm_crt(char transa, char transb, int64_t m, int64_t n, int64_t k,
                  double alpha, const double *A, int64_t lda,
                  const double *B, int64_t ldb,
                  double beta, double *C, int64_t ldc,
                  int nmoduli, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * The residue step alone, for one operand (operand, trans, rows, k, X, ld as for
 * mdg_split_slices): writes the symmetric residues of the `bits`-wide scaled integers modulo the
 * first nmoduli moduli, residue l of entry (r, p) at the byte mdg_split_slices gives slice l, and
 * the exponents (0x7FFFFFFF for a row holding NaN or Inf, whose residues are then zero). Returns 0,
 * or 1 operand, 2 trans, 3 rows < 0, 4 k < 0, 5 X NULL, 6 ld too small, 7 nmoduli out of range,
 * 8 bits outside 1..72, 9 output NULL, or a negative runtime code.
 */
int mdg_crt_residues(int operand, char trans, int64_t rows, int64_t k, const double *X, int64_t ld,
                     int nmoduli, int bits, int8_t *residues, int32_t *exponents, void *stream);

/* ------------------------------------------------------------------------------------------
 * Grouped launch: many independent dgemm operations (each exactly as mdg_dgemm) in one
 * persistent kernel. Not in the paper; a batching layer over the same operation.
 *
 * 1. mdg_grouped_plan (host only, no HIP call) validates every GEMM and writes a plan: one
 *    descriptor per GEMM (device pointers and sizes copied from `descs`) and the list of output
 *    tiles in schedule order. tile_class[i] (NULL = automatic: 1 when m < 48 or n < 48, else 0)
 *    picks the tile of GEMM i: 0 = 64x64 workgroup tile (the tile of variant
 *    "mfma_f64_64x64x16_w32x32"), 1 = 32x32 workgroup tile (variant "mfma_f64_32x32x16_w16x16"),
 *    2 = 32x32 wave tile (variant "wave_f64_64x64x8_w32x32": each wave computes its own tiles
 *    with no LDS or barrier; bitwise the result of that variant and of the "ring_" variants).
 *    Class 2 cannot be mixed with classes 0 and 1 in one plan (code 3). schedule:
 *    MDG_SCHEDULE_NATURAL (GEMM by GEMM) or MDG_SCHEDULE_LPT (tiles by decreasing cost, i.e. tile
 *    area times k). In a class-2 plan every GEMM goes to one XCD (LPT: by decreasing cost to the
 *    least loaded XCD; NATURAL: round-robin) and each XCD's waves walk its own tile sublist.
 * 2. The caller copies the plan bytes to device memory (16-byte aligned) and keeps them, and the
 *    matrices the descriptors point to, alive and unchanged while launches are pending.
 * 3. mdg_dgemm_grouped launches one persistent kernel of `grid` workgroups of 4 waves (0 = 4 per
 *    CU; rounded up to a multiple of 8, the XCD count) that walks the tile list. It allocates and
 *    clears nothing, so it may be captured in a graph and replayed; every replay recomputes
 *    C := alpha*op(A)*op(B) + beta*C for every GEMM.
 * GEMMs must not write overlapping C (not checked).
 * ------------------------------------------------------------------------------------------ */

#define MDG_SCHEDULE_NATURAL 0
#define MDG_SCHEDULE_LPT 1

typedef struct mdg_gemm_desc {
  char transa, transb;
  int64_t m, n, k;
  double alpha;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double beta;
  double *C;
  int64_t ldc;
} mdg_gemm_desc;

/* Number of tile classes accepted in tile_class[]. */
int mdg_grouped_tile_classes(void);

/* Bytes of the plan for these GEMMs and tile classes, or -1 (count < 0, NULL descs, bad class). */
int64_t mdg_grouped_plan_bytes(int count, const mdg_gemm_desc *descs, const int32_t *tile_class);

/*
 * Writes the plan into host memory `plan` (plan_bytes >= mdg_grouped_plan_bytes). Returns 0 and
 * the number of tiles in *num_tiles; or 1 bad count/descs, 3 bad tile class, 4 bad schedule,
 * 5 plan NULL or too small; or 100 + the mdg_dgemm argument code of the first invalid GEMM, whose
 * index goes to *bad_index; or MDG_ERR_SIZE.
 */
int mdg_grouped_plan(int count, const mdg_gemm_desc *descs, const int32_t *tile_class,
                     int schedule, void *plan, int64_t plan_bytes, int64_t *num_tiles,
                     int *bad_index);

/*
 * Runs a plan already in device memory. num_tiles is the value mdg_grouped_plan returned; grid is
 * the number of persistent workgroups (0 = four per CU; capped at num_tiles, then rounded up to a
 * multiple of 8). Returns 0, or
 * 1 plan NULL or misaligned, 2 num_tiles < 0, 3 grid < 0, or a negative runtime code.
 */
int mdg_dgemm_grouped(const void *device_plan, int64_t num_tiles, int grid, void *stream);

/* ------------------------------------------------------------------------------------------
 * Level-3 operations built on the GEMM (the paper's Step 2, "Poorman's BLAS": with a fast GEMM
 * on submatrices the other level-3 BLAS follow; Kagstrom, Ling and Van Loan). Definitions,
 * argument order and argument checks are those of the level-3 BLAS routines of the same names
 * (Dongarra, Du Croz, Hammarling and Duff, cited in the paper's section 1.1). Storage is
 * column-major with leading dimensions, as above; device pointers, caller-owned, no workspace,
 * asynchronous on `stream`. Return values as for mdg_dgemm: 0, the 1-based position of the first
 * bad argument, or a negative MDG_ERR_* code.
 * ------------------------------------------------------------------------------------------ */

/*
 * Symmetric rank-k update on one triangle of the n x n C:
 *
 *     C := alpha * op(A) * op(A)^T + beta * C,   op(A) = A (trans 'N', A stored n x k)
 *                                                or A^T (trans 'T', A stored k x n).
 *
 * uplo 'L' ('l'): the lower triangle (i >= j) is read and written; 'U': the upper (i <= j). The
 * other triangle is neither read nor written. One launch of the GEMM's ring kernels over the
 * tiles that meet the triangle, the epilogue masked to it; for n = 1024 * 2^j >= 4096 and
 * k >= 2048 the rectangles between diagonal blocks of order 1024 are computed first as GEMMs
 * (mdg_dgemm), and the one launch covers the diagonal blocks only. Checks: 1 uplo, 2 trans, 3 n < 0,
 * 4 k < 0, 6 A == NULL where read, 7 lda < max(1, rows of stored A), 9 C == NULL where touched,
 * 10 ldc < max(1, n). alpha == 0 or k == 0: A is not read and the triangle becomes beta*C
 * (beta == 0 writes zeros without reading C); n == 0, or that case with beta == 1: nothing is
 * enqueued. MDG_ERR_SIZE as for mdg_dgemm.
 */
int mdg_dsyrk(char uplo, char trans, int64_t n, int64_t k, double alpha, const double *A,
              int64_t lda, double beta, double *C, int64_t ldc, void *stream);

/*
 * The same with an explicit ring configuration, named by its GEMM variant id (or
 * MDG_VARIANT_AUTO). An explicit id always runs one launch over the whole triangle. Ids that
 * cannot run the given triangle return MDG_ERR_VARIANT. Integer-valued data give
 * bitwise-identical results in every accepted variant and in the automatic split.
 */
int mdg_dsyrk_ex(int variant, char uplo, char trans, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, double beta, double *C, int64_t ldc, void *stream);

/* The GEMM variant id of mdg_dsyrk's triangle launch for a product of this shape (for
 * n = 1024 * 2^j >= 4096 and k >= 2048 the launch over the diagonal blocks; host only), or
 * MDG_ERR_VARIANT for invalid flags or sizes. */
int mdg_dsyrk_select_variant(char uplo, char trans, int64_t n, int64_t k);

/*
 * Triangular matrix-matrix multiply, in place on the m x n B:
 *
 *     B := alpha * op(A) * B   (side 'L', A of order m)   or   B := alpha * B * op(A)   (side 'R',
 *     A of order n),
 *
 * A triangular: uplo 'L' or 'U' names the stored triangle that is read (the other is not), diag
 * 'U' takes the diagonal as ones without reading it ('N': read). transa 'N' or 'T'/'C'.
 * Computed by recursive halving of op(A): the off-diagonal blocks by mdg_dgemm, each diagonal
 * block of order <= 64 by one small kernel per block, all in order on `stream` (about 2m/64 or
 * 2n/64 launches). Checks: 1 side, 2 uplo, 3 transa, 4 diag, 5 m < 0, 6 n < 0, 8 A == NULL where
 * read, 9 lda < max(1, order of A), 10 B == NULL (m, n > 0), 11 ldb < max(1, m). Every GEMM of
 * the recursion is checked before the first launch (MDG_ERR_SIZE if one would be refused), so a
 * failed check enqueues nothing; an MDG_ERR_HIP from a later launch leaves B partly updated.
 * alpha == 0: B := 0 without reading A or B. m == 0 or n == 0: nothing is enqueued. A and B must
 * not overlap.
 */
int mdg_dtrmm(char side, char uplo, char transa, char diag, int64_t m, int64_t n, double alpha,
              const double *A, int64_t lda, double *B, int64_t ldb, void *stream);

/*
 * Triangular solve with many right-hand sides, X overwriting the m x n B:
 *
 *     op(A) * X = alpha * B   (side 'L')   or   X * op(A) = alpha * B   (side 'R'),
 *
 * with A, uplo, transa, diag, the checks, the launches and the error behaviour as for
 * mdg_dtrmm. The diagonal blocks are solved by substitution; there is no test for singularity (a
 * zero on a non-unit diagonal divides by zero, as in the reference BLAS).
 */
int mdg_dtrsm(char side, char uplo, char transa, char diag, int64_t m, int64_t n, double alpha,
              const double *A, int64_t lda, double *B, int64_t ldb, void *stream);

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

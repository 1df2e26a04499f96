// mdg_internal.h -- declarations shared by the library's source files (not part of the C ABI).
#ifndef MDG_INTERNAL_H
#define MDG_INTERNAL_H

#include <stdint.h>

// Records the raw hipError_t of a failed HIP call for mdg_last_hip_error() on this thread.
__attribute__((visibility("hidden"))) void mdg_record_hip_error(int err);

// What mdg_dgemm would return before its first HIP call for these arguments (0: it would
// enqueue work or return at once). No HIP call, no pointer dereference.
__attribute__((visibility("hidden"))) int mdg_dgemm_precheck(
    char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
    int64_t lda, const double* B, int64_t ldb, double beta, const double* C, int64_t ldc);

// The gfx950 check of the current device every entry point makes before enqueuing work:
// MDG_SUCCESS, MDG_ERR_DEVICE or MDG_ERR_HIP.
__attribute__((visibility("hidden"))) int mdg_device_check(void);

#endif

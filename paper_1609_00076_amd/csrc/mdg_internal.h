// mdg_internal.h -- declarations shared by the library's source files (not part of the C ABI).
#ifndef MDG_INTERNAL_H
#define MDG_INTERNAL_H

// Records the raw hipError_t of a failed HIP call for mdg_last_hip_error() on this thread.
__attribute__((visibility("hidden"))) void mdg_record_hip_error(int err);

#endif

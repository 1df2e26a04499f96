"""MI355X-native double-precision GEMM (dgemm) with hand-written gfx950 HIP kernels.

C := alpha*op(A)*op(B) + beta*C on column-major operands with leading
dimensions, and the level-3 operations built on it (dsyrk, dtrmm, dtrsm),
exported by libmdg.so through the C ABI in include/mdg.h. This
package is the thin Python binding (ctypes); torch supplies device memory and
streams only.
"""
from .binding import (MDG_ERR_DEVICE, MDG_ERR_HIP, MDG_ERR_SCRATCH, MDG_ERR_SIZE, MDG_ERR_VARIANT,
                      MDG_SCHEDULE_LPT, MDG_SCHEDULE_NATURAL, MdgError, dgemm, gemm2d, gemm2d_args, load,
                      mdg_crt_bits, mdg_crt_max_moduli, mdg_crt_residues, mdg_dgemm, mdg_dgemm_crt,
                      mdg_dgemm_crt_workspace_size,
                      mdg_dgemm_ex, mdg_dgemm_grouped, mdg_dgemm_plan, mdg_dgemm_split, mdg_dgemm_split_noalloc,
                      mdg_dgemm_split_noalloc_max_bytes, mdg_dsyrk,
                      mdg_dsyrk_ex, mdg_dsyrk_select_variant, mdg_dtrmm, mdg_dtrsm,
                      mdg_dgemm_split_workspace_size, mdg_gemm_desc, mdg_grouped_plan,
                      mdg_grouped_plan_bytes, mdg_grouped_tile_classes, mdg_last_hip_error,
                      mdg_num_variants, mdg_select_variant, mdg_split_max_slices,
                      mdg_split_slices, mdg_status_string, mdg_variant_info, mdg_variant_name,
                      mdg_version)

__all__ = ["MDG_ERR_DEVICE", "MDG_ERR_HIP", "MDG_ERR_SCRATCH", "MDG_ERR_SIZE", "MDG_ERR_VARIANT",
           "MDG_SCHEDULE_LPT", "MDG_SCHEDULE_NATURAL", "MdgError", "dgemm", "gemm2d", "gemm2d_args", "load",
           "mdg_crt_bits", "mdg_crt_max_moduli", "mdg_crt_residues", "mdg_dgemm", "mdg_dgemm_crt",
           "mdg_dgemm_crt_workspace_size",
           "mdg_dgemm_ex", "mdg_dgemm_grouped", "mdg_dgemm_plan", "mdg_dgemm_split", "mdg_dgemm_split_noalloc",
           "mdg_dgemm_split_noalloc_max_bytes", "mdg_dgemm_split_workspace_size",
           "mdg_dsyrk", "mdg_dsyrk_ex", "mdg_dsyrk_select_variant", "mdg_dtrmm", "mdg_dtrsm",
           "mdg_gemm_desc", "mdg_grouped_plan", "mdg_grouped_plan_bytes",
           "mdg_grouped_tile_classes", "mdg_last_hip_error", "mdg_num_variants",
           "mdg_select_variant", "mdg_split_max_slices", "mdg_split_slices", "mdg_status_string",
           "mdg_variant_info", "mdg_variant_name", "mdg_version"]

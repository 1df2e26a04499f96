"""Thin ctypes binding of libmdg.so (include/mdg.h); argument marshalling only.

Each ``mdg_*`` function here has the name, argument order and return code of
the C entry point of the same name. Matrix arguments may be torch tensors
(float64, on the HIP device; the pointer passed is ``data_ptr()``), raw device
addresses as ints, or None (NULL). For tensors the binding also checks, before
the call, that the storage from ``data_ptr()`` onward covers every element the
call may touch, so that a caller's mistake becomes an exception instead of an
out-of-bounds access on the GPU. All computation happens in the HIP kernels;
there is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

from .build import LIB_PATH

_lib = None

MDG_SCHEDULE_NATURAL = 0
MDG_SCHEDULE_LPT = 1
MDG_ERR_HIP = -1
MDG_ERR_VARIANT = -2
MDG_ERR_DEVICE = -3
MDG_ERR_SIZE = -4
MDG_ERR_SCRATCH = -5


class mdg_gemm_desc(ctypes.Structure):
    """One GEMM of a grouped launch (the C struct of the same name)."""
    _fields_ = [("transa", ctypes.c_char), ("transb", ctypes.c_char),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("beta", ctypes.c_double), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class MdgError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        detail = f" (hipError_t {mdg_last_hip_error()})" if status == -1 else ""
        super().__init__(f"mdg status {status}: {mdg_status_string(status)}{detail}")


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def load():
    """Open libmdg.so (built in-tree by paper_1609_00076_amd.build); raise if absent.

    torch is imported first so that the library binds to the HIP runtime torch
    already uses: torch wheels carry their own libamdhip64, and a second runtime
    in the same process cannot see torch's device memory or streams.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1609_00076_amd.build` "
                          "(or __graft_entry__.build()) first")
    import torch  # noqa: F401  (loads torch's HIP runtime before ours is resolved)
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped into this process (" + ", ".join(runtimes) +
                          "); libmdg.so must share torch's runtime")
    i64, dbl, vp, ch, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_char, ctypes.c_int
    gemm_args = [ch, ch, i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp]
    lib.mdg_dgemm.argtypes = gemm_args
    lib.mdg_dgemm.restype = ci
    lib.mdg_dgemm_ex.argtypes = [ci] + gemm_args
    lib.mdg_dgemm_ex.restype = ci
    lib.mdg_select_variant.argtypes = [ch, ch, i64, i64, i64, dbl, dbl]
    lib.mdg_select_variant.restype = ci
    lib.mdg_dgemm_plan.argtypes = [ch, ch, i64, i64, i64, ctypes.POINTER(ci),
                                   ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.mdg_dgemm_plan.restype = ci
    lib.mdg_num_variants.argtypes = []
    lib.mdg_num_variants.restype = ci
    lib.mdg_variant_name.argtypes = [ci]
    lib.mdg_variant_name.restype = ctypes.c_char_p
    lib.mdg_variant_info.argtypes = [ci] + [ctypes.POINTER(ci)] * 4
    lib.mdg_variant_info.restype = ci
    lib.mdg_status_string.argtypes = [ci]
    lib.mdg_status_string.restype = ctypes.c_char_p
    lib.mdg_version.argtypes = []
    lib.mdg_version.restype = ci
    lib.mdg_last_hip_error.argtypes = []
    lib.mdg_last_hip_error.restype = ci
    lib.mdg_split_max_slices.argtypes = []
    lib.mdg_split_max_slices.restype = ci
    lib.mdg_dgemm_split_workspace_size.argtypes = [i64, i64, i64, ci]
    lib.mdg_dgemm_split_workspace_size.restype = i64
    lib.mdg_dgemm_split.argtypes = gemm_args[:-1] + [ci, vp, i64, vp]
    lib.mdg_dgemm_split.restype = ci
    lib.mdg_dgemm_split_noalloc.argtypes = gemm_args[:-1] + [ci, vp]
    lib.mdg_dgemm_split_noalloc.restype = ci
    lib.mdg_dgemm_split_noalloc_max_bytes.argtypes = []
    lib.mdg_dgemm_split_noalloc_max_bytes.restype = i64
    lib.mdg_crt_max_moduli.argtypes = []
    lib.mdg_crt_max_moduli.restype = ci
    lib.mdg_crt_bits.argtypes = [i64, ci]
    lib.mdg_crt_bits.restype = ci
    lib.mdg_dgemm_crt_workspace_size.argtypes = [i64, i64, i64, ci]
    lib.mdg_dgemm_crt_workspace_size.restype = i64
    lib.mdg_dgemm_crt.argtypes = gemm_args[:-1] + [ci, vp, i64, vp]
    lib.mdg_dgemm_crt.restype = ci
    lib.mdg_crt_residues.argtypes = [ci, ch, i64, i64, vp, i64, ci, ci, vp, vp, vp]
    lib.mdg_crt_residues.restype = ci
    lib.mdg_split_slices.argtypes = [ci, ch, i64, i64, vp, i64, ci, vp, vp, vp]
    lib.mdg_split_slices.restype = ci
    dptr = ctypes.POINTER(mdg_gemm_desc)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.mdg_grouped_tile_classes.argtypes = []
    lib.mdg_grouped_tile_classes.restype = ci
    lib.mdg_grouped_plan_bytes.argtypes = [ci, dptr, i32p]
    lib.mdg_grouped_plan_bytes.restype = i64
    lib.mdg_grouped_plan.argtypes = [ci, dptr, i32p, ci, vp, i64, ctypes.POINTER(i64),
                                     ctypes.POINTER(ci)]
    lib.mdg_grouped_plan.restype = ci
    lib.mdg_dgemm_grouped.argtypes = [vp, i64, ci, vp]
    lib.mdg_dgemm_grouped.restype = ci
    syrk_args = [ch, ch, i64, i64, dbl, vp, i64, dbl, vp, i64, vp]
    lib.mdg_dsyrk.argtypes = syrk_args
    lib.mdg_dsyrk.restype = ci
    lib.mdg_dsyrk_ex.argtypes = [ci] + syrk_args
    lib.mdg_dsyrk_ex.restype = ci
    lib.mdg_dsyrk_select_variant.argtypes = [ch, ch, i64, i64]
    lib.mdg_dsyrk_select_variant.restype = ci
    for name in ("mdg_dtrmm", "mdg_dtrsm"):
        f = getattr(lib, name)
        f.argtypes = [ch, ch, ch, ch, i64, i64, dbl, vp, i64, vp, i64, vp]
        f.restype = ci
    _lib = lib
    return lib


def _ch(t) -> bytes:
    if isinstance(t, bytes):
        return t[:1]
    if isinstance(t, str) and len(t) == 1:
        return t.encode()
    return b"\0"  # rejected by the library's argument check


def _is_trans(t) -> bool:
    return _ch(t) in (b"T", b"t", b"C", b"c")


def _extent(rows: int, cols: int, ld: int) -> int:
    """Elements from the first one to the last one of a rows x cols column-major matrix."""
    return 0 if rows <= 0 or cols <= 0 else (cols - 1) * ld + rows


def _ptr(x, need: int, name: str):
    """Device address of x; for tensors, also check dtype, device and storage extent."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, an int address or None")
    if x.dtype != torch.float64:
        raise TypeError(f"{name}: dtype must be float64, got {x.dtype}")
    if x.device.type != "cuda":
        raise TypeError(f"{name}: tensor must be on the HIP device, got {x.device}")
    if need > 0:
        st = x.untyped_storage()
        avail = (st.data_ptr() + st.nbytes() - x.data_ptr()) // 8
        if avail < need:
            raise ValueError(f"{name}: storage holds {avail} doubles past data_ptr(), call needs {need}")
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # a torch.cuda.Stream


def _marshal(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream):
    empty = m <= 0 or n <= 0
    reads_ab = not empty and alpha != 0.0 and k > 0
    touches_c = not empty and not ((alpha == 0.0 or k <= 0) and beta == 1.0)
    ra, ca = (k, m) if _is_trans(transa) else (m, k)
    rb, cb = (n, k) if _is_trans(transb) else (k, n)
    need_a = _extent(ra, ca, lda) if reads_ab and lda >= max(1, ra) else 0
    need_b = _extent(rb, cb, ldb) if reads_ab and ldb >= max(1, rb) else 0
    need_c = _extent(m, n, ldc) if touches_c and ldc >= max(1, m) else 0
    return (_ch(transa), _ch(transb), int(m), int(n), int(k), float(alpha),
            _ptr(A, need_a, "A"), int(lda), _ptr(B, need_b, "B"), int(ldb), float(beta),
            _ptr(C, need_c, "C"), int(ldc), _stream(stream) if touches_c else None)


def mdg_dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None) -> int:
    """C := alpha*op(A)*op(B) + beta*C; returns the library's status code."""
    return load().mdg_dgemm(*_marshal(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                                      ldc, stream))


def mdg_dgemm_ex(variant, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                 stream=None) -> int:
    """mdg_dgemm with an explicit kernel variant (or -1 for automatic choice)."""
    return load().mdg_dgemm_ex(int(variant), *_marshal(transa, transb, m, n, k, alpha, A, lda, B,
                                                       ldb, beta, C, ldc, stream))


def _marshal_syrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream):
    reads_a = n > 0 and alpha != 0.0 and k > 0
    touches_c = n > 0 and not ((alpha == 0.0 or k <= 0) and beta == 1.0)
    ra, ca = (k, n) if _is_trans(trans) else (n, k)
    need_a = _extent(ra, ca, lda) if reads_a and lda >= max(1, ra) else 0
    need_c = _extent(n, n, ldc) if touches_c and ldc >= max(1, n) else 0
    return (_ch(uplo), _ch(trans), int(n), int(k), float(alpha), _ptr(A, need_a, "A"), int(lda),
            float(beta), _ptr(C, need_c, "C"), int(ldc), _stream(stream) if touches_c else None)


def mdg_dsyrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None) -> int:
    """C := alpha*op(A)*op(A)^T + beta*C on the `uplo` triangle of C."""
    return load().mdg_dsyrk(*_marshal_syrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream))


def mdg_dsyrk_ex(variant, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None) -> int:
    """mdg_dsyrk with the ring configuration of an explicit GEMM variant id (or -1)."""
    return load().mdg_dsyrk_ex(int(variant), *_marshal_syrk(uplo, trans, n, k, alpha, A, lda, beta,
                                                            C, ldc, stream))


def mdg_dsyrk_select_variant(uplo, trans, n, k) -> int:
    return load().mdg_dsyrk_select_variant(_ch(uplo), _ch(trans), int(n), int(k))


def _marshal_tri(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb, stream):
    empty = m <= 0 or n <= 0
    na = m if _ch(side) in (b"L", b"l") else n
    need_a = _extent(na, na, lda) if not empty and alpha != 0.0 and lda >= max(1, na) else 0
    need_b = _extent(m, n, ldb) if not empty and ldb >= max(1, m) else 0
    return (_ch(side), _ch(uplo), _ch(transa), _ch(diag), int(m), int(n), float(alpha),
            _ptr(A, need_a, "A"), int(lda), _ptr(B, need_b, "B"), int(ldb),
            None if empty else _stream(stream))


def mdg_dtrmm(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb, stream=None) -> int:
    """B := alpha*op(A)*B (side L) or alpha*B*op(A) (side R), A triangular."""
    return load().mdg_dtrmm(*_marshal_tri(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb,
                                          stream))


def mdg_dtrsm(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb, stream=None) -> int:
    """Solve op(A)*X = alpha*B (side L) or X*op(A) = alpha*B (side R); X overwrites B."""
    return load().mdg_dtrsm(*_marshal_tri(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb,
                                          stream))


def mdg_select_variant(transa, transb, m, n, k, alpha, beta) -> int:
    return load().mdg_select_variant(_ch(transa), _ch(transb), int(m), int(n), int(k),
                                     float(alpha), float(beta))


def mdg_dgemm_plan(transa, transb, m, n, k):
    """(variant, m_main, n_main) of the automatic dgemm: the tiled variant (or -1) covers rows
    [0, m_main) and columns [0, n_main) of C, the thin kernel the rest. Raises MdgError on an
    invalid argument."""
    v, mm, nn = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
    st = load().mdg_dgemm_plan(_ch(transa), _ch(transb), int(m), int(n), int(k), ctypes.byref(v),
                               ctypes.byref(mm), ctypes.byref(nn))
    if st:
        raise MdgError(st)
    return v.value, mm.value, nn.value


def mdg_num_variants() -> int:
    return load().mdg_num_variants()


def mdg_variant_name(variant: int):
    s = load().mdg_variant_name(int(variant))
    return None if s is None else s.decode()


def mdg_variant_info(variant: int):
    """(mt, nt, kt, threads) of a variant; raises MdgError for an unknown id."""
    vals = [ctypes.c_int() for _ in range(4)]
    st = load().mdg_variant_info(int(variant), *[ctypes.byref(v) for v in vals])
    if st:
        raise MdgError(st)
    return tuple(v.value for v in vals)


def mdg_status_string(status: int) -> str:
    return load().mdg_status_string(int(status)).decode()


def mdg_version() -> int:
    return load().mdg_version()


def mdg_last_hip_error() -> int:
    return load().mdg_last_hip_error()


def mdg_split_max_slices() -> int:
    return load().mdg_split_max_slices()


def mdg_dgemm_split_workspace_size(m, n, k, nslices) -> int:
    return load().mdg_dgemm_split_workspace_size(int(m), int(n), int(k), int(nslices))


def _raw_ptr(x, need_bytes: int, name: str):
    """Device address of a tensor of any dtype (storage extent checked in bytes), int or None."""
    if x is None or isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise TypeError(f"{name}: expected a device tensor, an int address or None")
    st = x.untyped_storage()
    if st.data_ptr() + st.nbytes() - x.data_ptr() < need_bytes:
        raise ValueError(f"{name}: storage smaller than the {need_bytes} bytes the call needs")
    return x.data_ptr()


def mdg_dgemm_split(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices,
                    workspace, workspace_bytes, stream=None) -> int:
    """Split-precision C := alpha*op(A)*op(B) + beta*C on INT8 MFMA; returns the status code.

    `workspace` is a device tensor (any dtype) or address of at least `workspace_bytes` bytes.
    """
    args = _marshal(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    ws = _raw_ptr(workspace, max(0, int(workspace_bytes)), "workspace")
    return load().mdg_dgemm_split(*args[:-1], int(nslices), ws, int(workspace_bytes), args[-1])


def mdg_dgemm_split_noalloc_max_bytes() -> int:
    return load().mdg_dgemm_split_noalloc_max_bytes()


def mdg_dgemm_split_noalloc(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                            nslices, stream=None) -> int:
    """mdg_dgemm_split on the library's static scratch array (no workspace, no allocation)."""
    args = _marshal(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    return load().mdg_dgemm_split_noalloc(*args[:-1], int(nslices), args[-1])


def mdg_split_slices(operand, trans, rows, k, X, ld, nslices, slices, exponents, stream=None) -> int:
    """Slicing step alone (operand 0: rows of op(A); 1: columns of op(B)); returns the status."""
    kp = (int(k) + 63) // 64 * 64
    row_contig = _is_trans(trans) if operand == 0 else not _is_trans(trans)
    need_x = _extent(k if row_contig else rows, rows if row_contig else k, ld) \
        if rows > 0 and k > 0 and ld >= max(1, k if row_contig else rows) else 0
    ok_s = 1 <= int(nslices) <= mdg_split_max_slices()
    xp = _ptr(X, need_x, "X")
    rp = (int(rows) + 127) // 128 * 128
    sp = _raw_ptr(slices, int(nslices) * rp * kp if ok_s and rows > 0 else 0, "slices")
    ep = _raw_ptr(exponents, 4 * int(rows) if rows > 0 else 0, "exponents")
    return load().mdg_split_slices(int(operand), _ch(trans), int(rows), int(k), xp, int(ld),
                                   int(nslices), sp, ep, _stream(stream))


def mdg_crt_max_moduli() -> int:
    return load().mdg_crt_max_moduli()


def mdg_crt_bits(k, nmoduli) -> int:
    return load().mdg_crt_bits(int(k), int(nmoduli))


def mdg_dgemm_crt_workspace_size(m, n, k, nmoduli) -> int:
    return load().mdg_dgemm_crt_workspace_size(int(m), int(n), int(k), int(nmoduli))


def mdg_dgemm_crt(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nmoduli,
                  workspace, workspace_bytes, stream=None) -> int:
    """Split-precision C := alpha*op(A)*op(B) + beta*C by the Chinese remainder theorem on INT8
    MFMA; `workspace` is a device tensor (any dtype) or address of at least `workspace_bytes`."""
    args = _marshal(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    ws = _raw_ptr(workspace, max(0, int(workspace_bytes)), "workspace")
    return load().mdg_dgemm_crt(*args[:-1], int(nmoduli), ws, int(workspace_bytes), args[-1])


def mdg_crt_residues(operand, trans, rows, k, X, ld, nmoduli, bits, residues, exponents,
                     stream=None) -> int:
    """The residue step alone for one operand (layout as mdg_split_slices, slice l = modulus l)."""
    kp = (int(k) + 63) // 64 * 64
    row_contig = _is_trans(trans) if operand == 0 else not _is_trans(trans)
    need_x = _extent(k if row_contig else rows, rows if row_contig else k, ld) \
        if rows > 0 and k > 0 and ld >= max(1, k if row_contig else rows) else 0
    ok_n = 1 <= int(nmoduli) <= mdg_crt_max_moduli()
    xp = _ptr(X, need_x, "X")
    rp = (int(rows) + 127) // 128 * 128
    rsp = _raw_ptr(residues, int(nmoduli) * rp * kp if ok_n and rows > 0 else 0, "residues")
    ep = _raw_ptr(exponents, 4 * int(rows) if rows > 0 else 0, "exponents")
    return load().mdg_crt_residues(int(operand), _ch(trans), int(rows), int(k), xp, int(ld),
                                   int(nmoduli), int(bits), rsp, ep, _stream(stream))


def mdg_grouped_tile_classes() -> int:
    return load().mdg_grouped_tile_classes()


def _descs_array(descs):
    arr = (mdg_gemm_desc * max(1, len(descs)))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def _classes_array(tile_class, count):
    if tile_class is None:
        return None
    arr = (ctypes.c_int32 * max(1, count))(*[int(c) for c in tile_class])
    return arr


def mdg_grouped_plan_bytes(descs, tile_class=None) -> int:
    """descs: sequence of mdg_gemm_desc; tile_class: per-GEMM classes or None (automatic)."""
    return load().mdg_grouped_plan_bytes(len(descs), _descs_array(descs),
                                         _classes_array(tile_class, len(descs)))


def mdg_grouped_plan(descs, tile_class, schedule, plan):
    """Write the plan into `plan` (a writable host buffer, e.g. a numpy uint8 array).

    Returns (status, num_tiles, bad_index).
    """
    import numpy as np
    buf = np.ascontiguousarray(plan)
    if buf is not plan or buf.dtype != np.uint8:
        raise TypeError("plan must be a contiguous numpy uint8 array")
    nt = ctypes.c_int64(0)
    bad = ctypes.c_int(-1)
    st = load().mdg_grouped_plan(len(descs), _descs_array(descs),
                                 _classes_array(tile_class, len(descs)), int(schedule),
                                 buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes,
                                 ctypes.byref(nt), ctypes.byref(bad))
    return st, nt.value, bad.value


def mdg_dgemm_grouped(device_plan, num_tiles, grid=0, stream=None) -> int:
    """Launch a plan held in device memory (tensor or address)."""
    dp = _raw_ptr(device_plan, 64, "device_plan")
    return load().mdg_dgemm_grouped(dp, int(num_tiles), int(grid), _stream(stream))


def dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None, variant=-1):
    """mdg_dgemm_ex that raises MdgError on a non-zero status."""
    st = mdg_dgemm_ex(variant, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    if st:
        raise MdgError(st)


def _layout(shape, strides, name):
    """(stored transposed?, ld) of a 2-D tensor whose elements are unit-stride along one dimension.

    A tensor of shape (r, c) with strides (1, ld) is the column-major r x c matrix with leading
    dimension ld; strides (ld, 1) make it the column-major c x r matrix (its transpose) with
    leading dimension ld. A dimension of size 1 places no constraint on its stride."""
    r, c = shape
    s0, s1 = strides
    if s0 == 1 or r <= 1:
        if c <= 1 or s1 >= max(1, r):
            return False, max(1, r) if c <= 1 else s1
    if s1 == 1 or c <= 1:
        if r <= 1 or s0 >= max(1, c):
            return True, max(1, c) if r <= 1 else s0
    raise ValueError(f"{name}: strides {tuple(strides)} of shape {tuple(shape)} are neither "
                     "column-major (1, ld >= rows) nor row-major (ld >= cols, 1)")


def gemm2d_args(a_shape, a_strides, b_shape, b_strides, c_shape, c_strides, transa="N",
                transb="N"):
    """The dgemm call (transa, transb, m, n, k, lda, ldb, ldc, swap) for 2-D operands given by
    shape and strides, each unit-stride along one dimension. op(A) is m x k, op(B) k x n, C m x n.
    A row-major operand is passed as the column-major storage of its transpose with the transpose
    flag flipped. A row-major C is computed as C^T = op(B)^T op(A)^T (swap True: the first operand
    of the call is B)."""
    ta, tb = _is_trans(transa), _is_trans(transb)
    if len(a_shape) != 2 or len(b_shape) != 2 or len(c_shape) != 2:
        raise ValueError("gemm2d takes 2-D tensors")
    m, k = (a_shape[1], a_shape[0]) if ta else tuple(a_shape)
    kb, n = (b_shape[1], b_shape[0]) if tb else tuple(b_shape)
    if kb != k or tuple(c_shape) != (m, n):
        raise ValueError(f"shapes do not match: op(A) {m}x{k}, op(B) {kb}x{n}, C {tuple(c_shape)}")
    a_t, lda = _layout(a_shape, a_strides, "A")
    b_t, ldb = _layout(b_shape, b_strides, "B")
    c_t, ldc = _layout(c_shape, c_strides, "C")
    fa, fb = ta != a_t, tb != b_t  # flag for the column-major storage actually passed
    if not c_t:
        return ("T" if fa else "N", "T" if fb else "N", m, n, k, lda, ldb, ldc, False)
    # C stored as C^T (n x m column-major): C^T = op(B)^T op(A)^T
    return ("N" if fb else "T", "N" if fa else "T", n, m, k, ldb, lda, ldc, True)


def gemm2d(A, B, C, alpha=1.0, beta=0.0, transa="N", transb="N", stream=None, variant=-1):
    """C := alpha*op(A)*op(B) + beta*C on 2-D float64 device tensors, each column-major
    (strides (1, ld)) or row-major (strides (ld, 1)), sizes and leading dimensions taken from the
    tensors (see gemm2d_args). Raises MdgError on a non-zero status; returns C."""
    ta, tb, m, n, k, lda, ldb, ldc, swap = gemm2d_args(
        tuple(A.shape), A.stride(), tuple(B.shape), B.stride(), tuple(C.shape), C.stride(),
        transa, transb)
    first, second = (B, A) if swap else (A, B)
    dgemm(ta, tb, m, n, k, alpha, first, lda, second, ldb, beta, C, ldc, stream=stream,
          variant=variant)
    return C

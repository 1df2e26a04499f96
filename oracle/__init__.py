"""Plain CPU oracle for double-precision GEMM and the level-3 operations built on it.

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product package never imports it, and it
imports nothing from the product package.

The arithmetic lives in ``oracle_dgemm.c`` (plain C, gcc, no FMA contraction):
``C := alpha*op(A)*op(B) + beta*C`` evaluated entry by entry as the paper's
definition (section 1.2 for the dgemm operation and its four transpose cases,
section 2.1 for the sum over p, section 2.3 for column-major storage); the
symmetric rank-k update, triangular multiply and triangular solve of Step 2's
"Poorman's BLAS" live in ``oracle_blas3.c``, written from the level-3 BLAS
definitions. This module only marshals numpy arrays into that library.

Arrays are 1-D float64 numpy arrays holding the column-major storage of a
matrix with a leading dimension, exactly as a BLAS caller would pass them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build

_default = None


def load_library(path: str):
    """Open an oracle shared library at `path` and declare its entry points."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_dgemm.restype = ctypes.c_int
    lib.oracle_dgemm.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                 ctypes.c_double, dp, i64, dp, i64,
                                 ctypes.c_double, dp, i64]
    lib.oracle_dgemm_absden.restype = ctypes.c_int
    lib.oracle_dgemm_absden.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                        ctypes.c_double, dp, i64, dp, i64,
                                        ctypes.c_double, dp, i64, dp, i64]
    lib.oracle_dgemm_dd.restype = ctypes.c_int
    lib.oracle_dgemm_dd.argtypes = lib.oracle_dgemm.argtypes
    lib.oracle_dsyrk.restype = ctypes.c_int
    lib.oracle_dsyrk.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, ctypes.c_double,
                                 dp, i64, ctypes.c_double, dp, i64]
    for name in ("oracle_dtrmm", "oracle_dtrsm"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_char, ctypes.c_char, i64, i64,
                      ctypes.c_double, dp, i64, dp, i64]
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_get_threads.argtypes = []
    return lib


def _load():
    global _default
    if _default is None:
        if not os.path.exists(LIB_PATH):
            build()
        _default = load_library(LIB_PATH)
    return _default


def _ptr(x):
    """Pointer to a float64 numpy array (None -> NULL)."""
    if x is None:
        return None
    if x.dtype != np.float64 or not x.flags["C_CONTIGUOUS"]:
        raise TypeError("oracle arrays must be contiguous float64")
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ch(t):
    return t.encode() if isinstance(t, str) else bytes([t])


def dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """C := alpha*op(A)*op(B) + beta*C in place on the flat column-major array C.

    Returns the status code (0, or the 1-based position of the first invalid
    argument as in the BLAS reference argument check).
    """
    return (lib or _load()).oracle_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha),
                                _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C), ldc)


def dgemm_dd(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """As dgemm, each entry in doubled precision (Dot2) and rounded once: the true-error
    reference, not the parity target."""
    return (lib or _load()).oracle_dgemm_dd(_ch(transa), _ch(transb), m, n, k, float(alpha),
                                   _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C), ldc)


def absden(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc, D, ldd, lib=None):
    """D(i,j) := |alpha| sum_p |op(A)(i,p)||op(B)(p,j)| + |beta||C0(i,j)|."""
    return (lib or _load()).oracle_dgemm_absden(_ch(transa), _ch(transb), m, n, k, float(alpha),
                                       _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C0), ldc,
                                       _ptr(D), ldd)


def dsyrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, lib=None):
    """C := alpha*op(A)*op(A)^T + beta*C on the `uplo` triangle of C (level-3 BLAS dsyrk)."""
    return (lib or _load()).oracle_dsyrk(_ch(uplo), _ch(trans), n, k, float(alpha), _ptr(A), lda,
                                         float(beta), _ptr(C), ldc)


def dtrmm(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb, lib=None):
    """B := alpha*op(A)*B (side L) or alpha*B*op(A) (side R), A triangular (level-3 BLAS dtrmm)."""
    return (lib or _load()).oracle_dtrmm(_ch(side), _ch(uplo), _ch(transa), _ch(diag), m, n,
                                         float(alpha), _ptr(A), lda, _ptr(B), ldb)


def dtrsm(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb, lib=None):
    """Solve op(A)*X = alpha*B (side L) or X*op(A) = alpha*B (side R) by substitution; X
    overwrites B (level-3 BLAS dtrsm)."""
    return (lib or _load()).oracle_dtrsm(_ch(side), _ch(uplo), _ch(transa), _ch(diag), m, n,
                                         float(alpha), _ptr(A), lda, _ptr(B), ldb)


def set_threads(n: int, lib=None) -> None:
    (lib or _load()).oracle_set_threads(int(n))


def get_threads(lib=None) -> int:
    return (lib or _load()).oracle_get_threads()

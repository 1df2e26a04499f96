"""Reference of the error-free splitting behind the split-precision GEMM (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU slicing kernel
byte for byte and to state what the slice products sum to. It shares nothing with
the HIP path.

The split-precision GEMM approximates the FP64 product op(A) op(B) by the
Ozaki scheme (Ozaki, Ogita, Oishi and Rump, "Error-free transformations of matrix
multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59, 2012; the integer form of Ootomo, Ozaki and
Yokota, "DGEMM on integer matrix multiplication unit", IJHPCA 2024), in this
order:

1. Scale each row i of op(A) by a power of two, 2^-e_i, where e_i is the binary
   exponent of the row's largest magnitude (max |a_i*| = f * 2^e_i with
   f in [0.5, 1)), so that every scaled entry lies in (-1, 1). A zero row has
   e_i = 0. Columns of op(B) are scaled the same way (exponents f_j).
2. Split each scaled entry x into S slices of beta = 7 bits: repeat S times
   x := 128 x, q := trunc(x), x := x - q, keeping q in [-127, 127]. Every step is
   exact in binary64 (a power-of-two scaling and the removal of an integer
   part), so x = sum_s q_s 2^(-7 s) + r 2^(-7 S) with |r| < 1.
3. Form the integer products P_st = A_s B_t (exact in int64 here; in int32 on
   the GPU while k * (pairs per diagonal) * 127^2 < 2^31) for the pairs with
   s + t <= S + 1.
4. Recombine in binary64 along the anti-diagonals d = s + t:
   C' = sum_d 2^(-7 d) * sum_{s+t=d} P_st, then unscale:
   C(i,j) = 2^(e_i + f_j) C'(i,j).

The result differs from the exact product by the dropped slice pairs and the
remainders, about k * 2^(-7 S) times the product of the row and column maxima.
"""
from __future__ import annotations

import numpy as np

BETA = 7


def row_exponents(X: np.ndarray) -> np.ndarray:
    """e_r with max_p |X[r, p]| = f * 2^e_r, f in [0.5, 1); 0 for an all-zero row."""
    mx = np.max(np.abs(X), axis=1) if X.shape[1] else np.zeros(X.shape[0])
    e = np.frexp(mx)[1].astype(np.int64)
    return np.where(mx == 0, 0, e)


def split_rows(X: np.ndarray, S: int):
    """Slices (list of S int8 arrays shaped like X) and row exponents of X (rows x k)."""
    e = row_exponents(X)
    R = np.ldexp(X, -e[:, None])
    out = []
    for _ in range(S):
        R = R * float(1 << BETA)
        q = np.trunc(R)
        out.append(q.astype(np.int8))
        R = R - q
    return out, e


def slice_product_sum(A: np.ndarray, B: np.ndarray, S: int) -> np.ndarray:
    """sum_{s+t <= S+1} 2^(-7(s+t)) A_s B_t, unscaled: the value the split GEMM forms
    (before alpha and beta) for dense op(A) (m x k) and op(B) (k x n)."""
    As, ea = split_rows(A, S)
    Bs, eb = split_rows(B.T, S)
    m, n = A.shape[0], B.shape[1]
    C = np.zeros((m, n))
    for d in range(2, S + 2):
        P = np.zeros((m, n), dtype=np.int64)
        for s in range(1, S + 1):
            t = d - s
            if 1 <= t <= S:
                P += As[s - 1].astype(np.int64) @ Bs[t - 1].astype(np.int64).T
        C += np.ldexp(P.astype(np.float64), -BETA * d)
    return np.ldexp(np.ldexp(C, ea[:, None]), eb[None, :])

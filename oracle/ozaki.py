"""Reference of the split-precision GEMM schemes (test infrastructure).

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


# ------------------------------------------------------------------------------------------------
# Scheme II: one integer product per modulus, recombined by the Chinese remainder theorem (Ozaki,
# Uchino and Imamura, "Ozaki Scheme II: A GEMM-oriented emulation of floating-point matrix
# multiplication using an integer modular technique", 2025), in this order:
#
# 1. Scale each row i of op(A) to integers of w bits: A'(i,p) = trunc(A(i,p) 2^(w - e_i)) with e_i
#    as above, so |A'| < 2^w; columns of op(B) the same way (exponents f_j).
# 2. Take N pairwise coprime moduli m_l <= 256 and, for each, the symmetric residues
#    a_l = A' mod m_l, b_l = B' mod m_l in [-128, 127] (int8).
# 3. Form P_l = a_l b_l exactly in integers (int32 on the GPU) and r_l = P_l mod m_l in [0, m_l).
# 4. Recombine: X is the unique integer with X = r_l (mod m_l) for all l and -M/2 <= X < M/2,
#    M = prod m_l. With w chosen so that 4 k 2^(2w) <= M, |A'B'| < M/2 and X = (A'B')(i,j) exactly.
# 5. C(i,j) = RN(X) 2^(e_i + f_j - 2w), RN the rounding of the integer X to binary64.
#
# The error against the exact product comes only from step 1 (each entry loses less than one unit
# of 2^(e_i - w) relative to its row's maximum) and from the one rounding in step 5.
# ------------------------------------------------------------------------------------------------
MODULI = (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191, 181, 179,
          173, 167, 163, 157, 151, 149)
MAX_BITS = 72


def crt_modulus(nmod: int) -> int:
    M = 1
    for m in MODULI[:nmod]:
        M *= m
    return M


def crt_bits(k: int, nmod: int) -> int:
    """The largest w <= 72 with 4 k 2^(2w) <= M (so every |A'B'| < M/2), or 0 if none."""
    M = crt_modulus(nmod)
    kk = max(1, k)
    w = 0
    while w < MAX_BITS and 4 * kk * (1 << (2 * (w + 1))) <= M:
        w += 1
    return w


def to_integers(X: np.ndarray, w: int):
    """(A' as a 2-D object array of Python ints, row exponents e): A'(r,p) = trunc(X 2^(w - e_r))."""
    e = row_exponents(X)
    S = np.ldexp(X, (w - e)[:, None])
    out = np.empty(X.shape, dtype=object)
    for idx, v in np.ndenumerate(S):
        out[idx] = int(np.trunc(v))
    return out, e


def sym_residue(x: int, m: int) -> int:
    """x mod m in [-(m // 2), m - m // 2 - 1]: [-128, 127] for m = 256, [-(m-1)/2, (m-1)/2] for odd m."""
    r = x % m
    return r - m if r >= m - m // 2 else r


def crt_residue_matrices(Xint: np.ndarray, nmod: int):
    """int8-valued residues (int64 arrays) of an integer matrix for the first nmod moduli."""
    f = np.vectorize(lambda v, m: sym_residue(int(v), m), otypes=[np.int64])
    return [f(Xint, m) for m in MODULI[:nmod]]


def crt_reconstruct(residues, nmod: int):
    """The signed integer matrix X with X = residues[l] (mod m_l) and -M/2 <= X < M/2."""
    M = crt_modulus(nmod)
    shape = residues[0].shape
    X = np.empty(shape, dtype=object)
    weights = []
    for m in MODULI[:nmod]:
        Ml = M // m
        weights.append(Ml * pow(Ml % m, -1, m))
    for idx in np.ndindex(*shape):
        s = sum(int(r[idx]) * wt for r, wt in zip(residues, weights)) % M
        X[idx] = s - M if s >= M // 2 else s
    return X


def crt_product(A: np.ndarray, B: np.ndarray, nmod: int):
    """Steps 1-4 for dense op(A) (m x k) and op(B) (k x n): (X, e, f, w)."""
    k = A.shape[1]
    w = crt_bits(k, nmod)
    Ai, ea = to_integers(A, w)
    Bi, eb = to_integers(B.T, w)
    ra = crt_residue_matrices(Ai, nmod)
    rb = crt_residue_matrices(Bi, nmod)
    prods = []
    for a, b, m in zip(ra, rb, MODULI[:nmod]):
        P = a @ b.T  # int64: |P| <= k 128^2
        prods.append(P % m)
    return crt_reconstruct(prods, nmod), ea, eb, w


def crt_emulated(A: np.ndarray, B: np.ndarray, nmod: int) -> np.ndarray:
    """Step 5: RN(X) 2^(e_i + f_j - 2w), the value the CRT split GEMM forms before alpha and beta."""
    X, ea, eb, w = crt_product(A, B, nmod)
    Xf = np.vectorize(float, otypes=[np.float64])(X)
    return np.ldexp(Xf, ea[:, None] + eb[None, :] - 2 * w)

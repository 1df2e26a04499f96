"""Seeded synthetic inputs for double-precision GEMM.

This module holds no GEMM arithmetic: it only draws matrices (and, for the
batched and served workloads, problem shapes) from numpy's PCG64 generator, in
column-major storage with a leading dimension, and fills the storage padding
with sentinels. Both the oracle tests and the GPU tests and benchmark draw from
it, so that both sides see the same bits.

Recipe:
  * a matrix with `rows` x `cols` logical entries and leading dimension `ld`
    is stored as a flat float64 array of ld*cols entries (entry (i,j) at
    j*ld + i, paper section 2.3);
  * values are drawn for the whole ld*cols storage in storage order, then the
    padding rows rows..ld-1 of every column are overwritten by a sentinel
    (quiet NaN for A and B, a signalling-NaN bit pattern for C), so a kernel
    that reads or writes padding is caught;
  * seeds are SEED_BASE + 1000*workload + 10*variant + matrix_id, with
    matrix_id 0 for A, 1 for B, 2 for C (and 3.. for probe vectors).
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 160900076

# Signalling NaN (quiet bit clear, payload non-zero): marks C padding rows.
PAD_C_BITS = 0x7FF0DEAD0000BEEF
PAD_AB = float("nan")


def pad_c_value() -> np.float64:
    return np.array([PAD_C_BITS], dtype=np.uint64).view(np.float64)[0]


def seed_for(workload: int, variant: int, matrix_id: int) -> int:
    return SEED_BASE + 1000 * workload + 10 * variant + matrix_id


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def is_trans(t: str) -> bool:
    if t in ("N", "n"):
        return False
    if t in ("T", "t", "C", "c"):
        return True
    raise ValueError(f"bad trans flag {t!r}")


def stored_dims(trans: str, rows_op: int, cols_op: int):
    """(rows, cols) of the stored array whose op() is rows_op x cols_op."""
    return (cols_op, rows_op) if is_trans(trans) else (rows_op, cols_op)


def ld_round8(rows: int) -> int:
    """Leading dimension = stored rows rounded up to a multiple of 8 (at least 8)."""
    return max(8, -(-rows // 8) * 8)


def ld_tight(rows: int) -> int:
    return max(1, rows)


def draw(gen: np.random.Generator, size: int, dist: str, phi: int = 0) -> np.ndarray:
    """`size` values in storage order from distribution `dist`.

    uniform: iid Uniform[-1, 1)
    int:     iid uniform integers in {-8, ..., 8} (exact products and sums)
    scaled:  u * 2**e with u ~ Uniform[-1, 1) and e ~ uniform integer in [-phi, phi]
    ones:    all 1.0
    zeros:   all 0.0
    """
    if dist == "uniform":
        return gen.uniform(-1.0, 1.0, size)
    if dist == "int":
        return gen.integers(-8, 9, size).astype(np.float64)
    if dist == "scaled":
        u = gen.uniform(-1.0, 1.0, size)
        e = gen.integers(-phi, phi + 1, size)
        return np.ldexp(u, e)
    if dist == "ones":
        return np.ones(size)
    if dist == "zeros":
        return np.zeros(size)
    raise ValueError(f"unknown distribution {dist!r}")


def matrix(seed: int, rows: int, cols: int, ld: int, dist: str = "uniform",
           phi: int = 0, pad=PAD_AB) -> np.ndarray:
    """Flat column-major storage (ld*cols float64) of a seeded rows x cols matrix."""
    if ld < max(1, rows):
        raise ValueError("ld < rows")
    x = draw(rng(seed), ld * cols, dist, phi)
    if ld > rows and cols > 0:
        x.reshape(cols, ld)[:, rows:] = pad
    return x


def view2d(x: np.ndarray, rows: int, cols: int, ld: int) -> np.ndarray:
    """The logical rows x cols matrix inside flat column-major storage (a view)."""
    return x.reshape(cols, ld)[:, :rows].T if cols > 0 else np.zeros((rows, 0))


def problem(workload: int, variant: int, transa: str, transb: str, m: int, n: int, k: int,
            ld_rule=ld_round8, dist: str = "uniform", phi: int = 0, c_dist=None):
    """Seeded operands of C := alpha*op(A)*op(B) + beta*C.

    Returns a dict with flat arrays A, B, C and leading dimensions lda, ldb, ldc
    (ld_rule applied to the rows of each stored array).
    """
    ra, ca = stored_dims(transa, m, k)
    rb, cb = stored_dims(transb, k, n)
    lda, ldb, ldc = ld_rule(ra), ld_rule(rb), ld_rule(m)
    A = matrix(seed_for(workload, variant, 0), ra, ca, lda, dist, phi)
    B = matrix(seed_for(workload, variant, 1), rb, cb, ldb, dist, phi)
    C = matrix(seed_for(workload, variant, 2), m, n, ldc, c_dist or dist, phi, pad=pad_c_value())
    return dict(transa=transa, transb=transb, m=m, n=n, k=k,
                A=A, lda=lda, B=B, ldb=ldb, C=C, ldc=ldc)


def log_uniform_int(gen: np.random.Generator, lo: int, hi: int, size) -> np.ndarray:
    """floor(exp(U[ln lo, ln(hi+1)))) clipped to [lo, hi]."""
    x = np.floor(np.exp(gen.uniform(math.log(lo), math.log(hi + 1), size))).astype(np.int64)
    return np.clip(x, lo, hi)


def triangular(seed: int, order: int, ld: int, uplo: str, dist: str = "uniform",
               unit: bool = False) -> np.ndarray:
    """Flat storage of a seeded order x order triangular matrix for dtrmm / dtrsm.

    The triangle named by `uplo` holds the values; every entry of the other triangle and of the
    padding rows is a quiet NaN, and with `unit` so is the diagonal (none of them may be read).
    uniform: off-diagonal Uniform[-1, 1) / order, diagonal of magnitude Uniform[1, 2) with a
             random sign (a well-conditioned triangle)
    int:     off-diagonal integers in {-4, ..., 4}, diagonal in {-4, -2, -1, 1, 2, 4} (so that a
             solve with integer right-hand sides built as op(A) X0 is exact)
    """
    g = rng(seed)
    x = np.full(ld * max(order, 1), PAD_AB)
    if order == 0:
        return x
    if dist == "uniform":
        vals = g.uniform(-1.0, 1.0, (order, order)) / order
        diag = g.uniform(1.0, 2.0, order) * np.where(g.random(order) < 0.5, -1.0, 1.0)
    elif dist == "int":
        vals = g.integers(-4, 5, (order, order)).astype(np.float64)
        diag = g.choice(np.array([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0]), order)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    np.fill_diagonal(vals, diag)
    keep = np.tril(np.ones((order, order), bool)) if uplo in "Ll" else np.triu(np.ones((order, order), bool))
    if unit:
        np.fill_diagonal(keep, False)
    vals[~keep] = PAD_AB
    x.reshape(order, ld)[:, :order] = vals.T
    return x


def grouped_batch(count: int = 2048, lo: int = 16, hi: int = 512, seed_variant: int = 0,
                  dist: str = "uniform"):
    """The batched workload: `count` independent GEMMs whose m, n, k are log-uniform integers in
    [lo, hi], transposes iid, alpha and beta ~ U[-1, 1), tight leading dimensions and entries
    drawn from `dist`. Returns a list of problem dicts (as `problem`) with alpha and beta added.
    With dist="int" the scalars are rounded to multiples of 0.5 so every result stays exact."""
    g = rng(seed_for(4, seed_variant, 9))
    m = log_uniform_int(g, lo, hi, count)
    n = log_uniform_int(g, lo, hi, count)
    k = log_uniform_int(g, lo, hi, count)
    ta = g.integers(0, 2, count)
    tb = g.integers(0, 2, count)
    ab = g.uniform(-1.0, 1.0, (count, 2))
    probs = []
    for i in range(count):
        p = problem(4, seed_variant * 10000 + i, "NT"[ta[i]], "NT"[tb[i]], int(m[i]), int(n[i]),
                    int(k[i]), ld_rule=ld_tight, dist=dist)
        alpha, beta = float(ab[i, 0]), float(ab[i, 1])
        if dist == "int":
            alpha, beta = float(np.round(alpha * 4) / 2), float(np.round(beta * 4) / 2)
        p["alpha"], p["beta"] = alpha, beta
        probs.append(p)
    return probs

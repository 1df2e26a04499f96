"""Pins of the oracle's level-3 routines (oracle_dsyrk, oracle_dtrmm, oracle_dtrsm)
to facts that do not come from the oracle itself.

Each pin takes an oracle library handle (None = the built oracle) and raises
AssertionError on a mismatch; test_oracle_blas3.py runs them and
test_oracle_mutants.py re-runs them against broken builds.

What pins what:
  library       scipy's LAPACK-backed BLAS (dsyrk, dtrmm, dtrsm) on random data, every
                flag combination, within a dot-product bound (syrk, trmm) or the
                forward-error bound of a well-conditioned solve (trsm)
  integer_exact integer-valued data: numpy int64 products with the triangle written out
                as a dense matrix, bitwise; for trsm, B = op(A) X0 with X0 integer and
                the diagonal powers of two, so substitution must return X0 exactly
  closed_forms  all-ones triangles: op(A) B is a running sum down the columns (left)
                or along the rows (right), from the top or the bottom according to the
                triangle; solving undoes it with first differences; syrk of all-ones
                data is alpha*k + beta*C0
  untouched     only the named triangle of A is read (NaN in the other one and, for a
                unit diagonal, on the diagonal), syrk writes only its triangle, and the
                padding rows of B and C keep their bits
  zero_rules    alpha = 0 sets B to zero without reading A or B; syrk with beta = 0
                ignores C0, with alpha = 0 or k = 0 and beta = 1 touches nothing
  threads       bitwise independence of the OpenMP thread count
  validation    argument-check codes in level-3 BLAS argument order
"""
import itertools

import numpy as np
import scipy.linalg.blas as sblas

import oracle

SIDES, UPLOS, TRANS, DIAGS = "LR", "LU", "NT", "NU"
COMBOS = list(itertools.product(SIDES, UPLOS, TRANS, DIAGS))


def _gamma(n):
    u = 2.0 ** -53
    return n * u / (1 - n * u)


def _store(M, ld, fill=np.nan):
    """Flat column-major storage of the 2-D array M with leading dimension ld; the padding
    rows hold `fill`."""
    rows, cols = M.shape
    S = np.full((max(cols, 1), ld), fill)
    S[:cols, :rows] = M.T
    return S.ravel().copy()


def _load(flat, rows, cols, ld):
    return flat.reshape(max(cols, 1), ld)[:cols, :rows].T.copy()


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


def _same(x, y):
    return np.array_equal(_bits(x), _bits(y))


def _tri_dense(Astored, uplo, transa, diag):
    """op(A) as a dense matrix: the named triangle of the stored A, the diagonal set to one
    when unit, transposed for 'T'."""
    T = np.tril(Astored) if uplo == "L" else np.triu(Astored)
    if diag == "U":
        np.fill_diagonal(T, 1.0)
    return T.T.copy() if transa == "T" else T


def _poison_other(Astored, uplo, diag):
    """The stored A with NaN in the triangle that must not be read (and on the diagonal when
    it is taken as one)."""
    A = Astored.copy()
    mask = np.triu(np.ones(A.shape, bool), 1) if uplo == "L" else np.tril(np.ones(A.shape, bool), -1)
    A[mask] = np.nan
    if diag == "U":
        np.fill_diagonal(A, np.nan)
    return A


def _tri_call(lib, fn, side, uplo, transa, diag, alpha, A, B, lda_pad=2, ldb_pad=3):
    """Run oracle dtrmm/dtrsm on 2-D A (na x na) and B (m x n); returns (status, B', flat B')."""
    m, n = B.shape
    na = A.shape[0]
    lda, ldb = na + lda_pad, max(m, 1) + ldb_pad
    fa, fb = _store(A, lda), _store(B, ldb)
    st = fn(side, uplo, transa, diag, m, n, alpha, fa, lda, fb, ldb, lib=lib)
    return st, _load(fb, m, n, ldb), fb


def _wellcond(g, na):
    """A triangular-ready matrix whose triangles are well conditioned: diagonal entries of
    magnitude in [1, 2], off-diagonal entries U[-1, 1] / na."""
    A = g.uniform(-1, 1, (na, na)) / na
    d = g.uniform(1, 2, na) * np.where(g.random(na) < 0.5, -1.0, 1.0)
    np.fill_diagonal(A, d)
    return A


def pin_blas3_library(lib=None):
    g = np.random.default_rng(31)
    for side, uplo, transa, diag in COMBOS:
        for (m, n) in ((37, 23), (5, 41), (64, 1)):
            na = m if side == "L" else n
            A = _wellcond(g, na)
            B = g.uniform(-1, 1, (m, n))
            alpha = 0.75
            kw = dict(side=int(side == "R"), lower=int(uplo == "L"), trans_a=int(transa == "T"),
                      diag=int(diag == "U"))
            T = _tri_dense(A, uplo, transa, diag)
            st, got, _ = _tri_call(lib, oracle.dtrmm, side, uplo, transa, diag, alpha, A, B)
            assert st == 0
            want = sblas.dtrmm(alpha, np.asfortranarray(A), np.asfortranarray(B), **kw)
            D = abs(alpha) * (np.abs(T) @ np.abs(B) if side == "L" else np.abs(B) @ np.abs(T))
            assert np.all(np.abs(got - want) <= 2 * _gamma(na + 2) * D + 1e-300), \
                ("trmm", side, uplo, transa, diag, m, n)
            st, got, _ = _tri_call(lib, oracle.dtrsm, side, uplo, transa, diag, alpha, A, B)
            assert st == 0
            want = sblas.dtrsm(alpha, np.asfortranarray(A), np.asfortranarray(B), **kw)
            scale = np.max(np.abs(want))
            assert np.max(np.abs(got - want)) <= 1e-13 * scale, ("trsm", side, uplo, transa, diag)
    for uplo, trans in itertools.product(UPLOS, TRANS):
        for n, k in ((33, 17), (8, 70), (50, 1)):
            A = g.uniform(-1, 1, (n, k) if trans == "N" else (k, n))
            C0 = g.uniform(-1, 1, (n, n))
            alpha, beta = -1.25, 0.5
            ld = A.shape[0] + 3
            fc = _store(C0, n + 2)
            st = oracle.dsyrk(uplo, trans, n, k, alpha, _store(A, ld), ld, beta, fc, n + 2, lib=lib)
            assert st == 0
            got = _load(fc, n, n, n + 2)
            want = sblas.dsyrk(alpha, np.asfortranarray(A), beta=beta, c=np.asfortranarray(C0),
                               trans=int(trans == "T"), lower=int(uplo == "L"))
            opA = A if trans == "N" else A.T
            D = abs(alpha) * (np.abs(opA) @ np.abs(opA).T) + abs(beta) * np.abs(C0)
            tri = np.tril(np.ones((n, n), bool)) if uplo == "L" else np.triu(np.ones((n, n), bool))
            assert np.all(np.abs(got - want)[tri] <= 2 * _gamma(k + 2) * D[tri]), ("syrk", uplo, trans)
            assert _same(got[~tri], C0[~tri]), ("syrk other triangle", uplo, trans)


def pin_blas3_integer_exact(lib=None):
    g = np.random.default_rng(32)
    for side, uplo, transa, diag in COMBOS:
        m, n = (29, 13) if side == "L" else (13, 29)
        na = m if side == "L" else n
        A = g.integers(-4, 5, (na, na)).astype(np.float64)
        np.fill_diagonal(A, g.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], na))
        T = _tri_dense(A, uplo, transa, diag)
        Ti = T.astype(np.int64)
        B = g.integers(-8, 9, (m, n)).astype(np.float64)
        Bi = B.astype(np.int64)
        st, got, _ = _tri_call(lib, oracle.dtrmm, side, uplo, transa, diag, 2.0, A, B)
        assert st == 0
        want = 2 * (Ti @ Bi if side == "L" else Bi @ Ti)
        assert _same(got, want.astype(np.float64)), ("trmm", side, uplo, transa, diag)
        # op(A) X0 = alpha B with alpha = 1/2: B = 2 op(A) X0 (exact integers); solving must give X0.
        X0 = Bi
        rhs = 2 * (Ti @ X0 if side == "L" else X0 @ Ti)
        st, got, _ = _tri_call(lib, oracle.dtrsm, side, uplo, transa, diag, 0.5, A,
                               rhs.astype(np.float64))
        assert st == 0
        # Values, not bits: a zero solution entry takes the sign of its last division.
        assert np.array_equal(got, X0.astype(np.float64)), ("trsm", side, uplo, transa, diag)
    for uplo, trans in itertools.product(UPLOS, TRANS):
        n, k = 21, 34
        A = g.integers(-8, 9, (n, k) if trans == "N" else (k, n))
        C0 = g.integers(-8, 9, (n, n))
        opA = A if trans == "N" else A.T
        full = 3 * (opA @ opA.T) - 2 * C0
        fc = _store(C0.astype(np.float64), n)
        st = oracle.dsyrk(uplo, trans, n, k, 1.5, _store(A.astype(np.float64), A.shape[0]),
                          A.shape[0], -1.0, fc, n, lib=lib)
        assert st == 0
        got = _load(fc, n, n, n)
        tri = np.tril(np.ones((n, n), bool)) if uplo == "L" else np.triu(np.ones((n, n), bool))
        assert _same(got[tri], (full[tri] / 2).astype(np.float64)), ("syrk", uplo, trans)


def pin_blas3_closed_forms(lib=None):
    m, n = 9, 6
    g = np.random.default_rng(33)
    B = g.integers(-9, 10, (m, n)).astype(np.float64)
    for side, uplo, transa, diag in COMBOS:
        na = m if side == "L" else n
        A = np.ones((na, na))
        op_lower = (uplo == "L") != (transa == "T")
        # op(A) lower ones on the left: running sums from the top; upper: from the bottom.
        # On the right, B*L sums each row from its right end, B*U from its left end.
        if side == "L":
            want = np.cumsum(B, 0) if op_lower else np.cumsum(B[::-1], 0)[::-1]
        else:
            want = np.cumsum(B[:, ::-1], 1)[:, ::-1] if op_lower else np.cumsum(B, 1)
        st, got, _ = _tri_call(lib, oracle.dtrmm, side, uplo, transa, diag, 1.0,
                               _poison_other(A, uplo, diag), B)
        assert st == 0 and _same(got, want), ("trmm ones", side, uplo, transa, diag)
        st, got, _ = _tri_call(lib, oracle.dtrsm, side, uplo, transa, diag, 1.0,
                               _poison_other(A, uplo, diag), want)
        assert st == 0 and _same(got, B), ("trsm ones", side, uplo, transa, diag)
    for uplo, trans in itertools.product(UPLOS, TRANS):
        nn, k = 7, 11
        C0 = g.integers(-9, 10, (nn, nn)).astype(np.float64)
        fc = _store(C0, nn + 1)
        A = np.ones((nn, k) if trans == "N" else (k, nn))
        st = oracle.dsyrk(uplo, trans, nn, k, 0.5, _store(A, A.shape[0]), A.shape[0], 2.0, fc,
                          nn + 1, lib=lib)
        got = _load(fc, nn, nn, nn + 1)
        tri = np.tril(np.ones((nn, nn), bool)) if uplo == "L" else np.triu(np.ones((nn, nn), bool))
        assert st == 0 and _same(got[tri], 0.5 * k + 2.0 * C0[tri]), ("syrk ones", uplo, trans)


def pin_blas3_untouched(lib=None):
    g = np.random.default_rng(34)
    for side, uplo, transa, diag in COMBOS:
        m, n = 11, 7
        na = m if side == "L" else n
        A = _wellcond(g, na)
        B = g.uniform(-1, 1, (m, n))
        for fn in (oracle.dtrmm, oracle.dtrsm):
            _, clean, _ = _tri_call(lib, fn, side, uplo, transa, diag, 1.5, A, B)
            st, got, flat = _tri_call(lib, fn, side, uplo, transa, diag, 1.5,
                                      _poison_other(A, uplo, diag), B)
            assert st == 0 and _same(got, clean), (fn.__name__, side, uplo, transa, diag)
            pad = flat.reshape(n, m + 3)[:, m:]
            assert np.all(np.isnan(pad)), "padding rows of B were written"
    for uplo, trans in itertools.product(UPLOS, TRANS):
        n, k = 9, 5
        A = g.uniform(-1, 1, (n, k) if trans == "N" else (k, n))
        C0 = g.uniform(-1, 1, (n, n))
        tri = np.tril(np.ones((n, n), bool)) if uplo == "L" else np.triu(np.ones((n, n), bool))
        C0[~tri] = np.nan
        fc = _store(C0, n + 2, fill=-7.0)
        st = oracle.dsyrk(uplo, trans, n, k, 1.0, _store(A, A.shape[0]), A.shape[0], 1.0, fc,
                          n + 2, lib=lib)
        got = _load(fc, n, n, n + 2)
        assert st == 0 and not np.any(np.isnan(got[tri])) and _same(got[~tri], C0[~tri])
        assert np.all(fc.reshape(n, n + 2)[:, n:] == -7.0), "padding rows of C were written"


def pin_blas3_zero_rules(lib=None):
    m, n = 6, 5
    for fn in (oracle.dtrmm, oracle.dtrsm):
        for side in SIDES:
            fb = np.full(m * n, np.nan)
            st = fn(side, "L", "N", "N", m, n, 0.0, None, m if side == "L" else n, fb, m, lib=lib)
            assert st == 0 and _same(fb, np.zeros(m * n)), (fn.__name__, side)
            fb = np.full(1, 3.0)
            assert fn(side, "U", "T", "U", 0, 4, 1.0, None, 4, fb, 1, lib=lib) == 0 and fb[0] == 3.0
    g = np.random.default_rng(35)
    A = g.uniform(-1, 1, (n, 3))
    C0 = np.full((n, n), np.nan)
    fc = _store(C0, n)
    assert oracle.dsyrk("L", "N", n, 3, 2.0, _store(A, n), n, 0.0, fc, n, lib=lib) == 0
    got = _load(fc, n, n, n)
    want = 2.0 * (A @ A.T)
    tri = np.tril(np.ones((n, n), bool))
    assert not np.any(np.isnan(got[tri])) and np.allclose(got[tri], want[tri], rtol=1e-14, atol=0)
    for alpha, k in ((0.0, 3), (1.0, 0)):
        C1 = g.uniform(-1, 1, (n, n))
        fc = _store(C1, n)
        assert oracle.dsyrk("U", "T", n, k, alpha, None, max(k, 1), 1.0, fc, n, lib=lib) == 0
        assert _same(_load(fc, n, n, n), C1)
        fc = _store(C1, n)
        assert oracle.dsyrk("U", "T", n, k, alpha, None, max(k, 1), -2.0, fc, n, lib=lib) == 0
        tri = np.triu(np.ones((n, n), bool))
        got = _load(fc, n, n, n)
        assert _same(got[tri], -2.0 * C1[tri]) and _same(got[~tri], C1[~tri])


def pin_blas3_threads(lib=None):
    g = np.random.default_rng(36)
    A = _wellcond(g, 40)
    B = g.uniform(-1, 1, (40, 33))
    out = []
    for t in (1, 5):
        oracle.set_threads(t, lib=lib)
        r = [_tri_call(lib, fn, s, "U", "T", "N", 0.5, A if s == "L" else A[:33, :33], B)[1]
             for fn in (oracle.dtrmm, oracle.dtrsm) for s in SIDES]
        fc = _store(B[:33, :33].copy(), 33)
        oracle.dsyrk("L", "N", 33, 40, 1.0, _store(B.T.copy(), 33), 33, 1.0, fc, 33, lib=lib)
        out.append(r + [fc])
    oracle.set_threads(0, lib=lib)
    assert all(_same(x, y) for x, y in zip(*out))


def pin_blas3_validation(lib=None):
    b = np.zeros(64)
    a = np.zeros(64)
    for fn in (oracle.dtrmm, oracle.dtrsm):
        assert fn("X", "L", "N", "N", 2, 2, 1.0, a, 2, b, 2, lib=lib) == 1
        assert fn("L", "X", "N", "N", 2, 2, 1.0, a, 2, b, 2, lib=lib) == 2
        assert fn("L", "L", "X", "N", 2, 2, 1.0, a, 2, b, 2, lib=lib) == 3
        assert fn("L", "L", "N", "X", 2, 2, 1.0, a, 2, b, 2, lib=lib) == 4
        assert fn("L", "L", "N", "N", -1, 2, 1.0, a, 2, b, 2, lib=lib) == 5
        assert fn("L", "L", "N", "N", 2, -1, 1.0, a, 2, b, 2, lib=lib) == 6
        assert fn("L", "L", "N", "N", 2, 2, 1.0, None, 2, b, 2, lib=lib) == 8
        assert fn("L", "L", "N", "N", 4, 2, 1.0, a, 3, b, 4, lib=lib) == 9   # lda < m on the left
        assert fn("R", "L", "N", "N", 4, 2, 1.0, a, 2, b, 4, lib=lib) == 0   # lda >= n on the right
        assert fn("R", "L", "N", "N", 2, 4, 1.0, a, 3, b, 2, lib=lib) == 9   # lda < n on the right
        assert fn("L", "L", "N", "N", 2, 2, 1.0, a, 2, None, 2, lib=lib) == 10
        assert fn("R", "L", "N", "N", 4, 2, 1.0, a, 4, b, 3, lib=lib) == 11  # ldb < m
    f = oracle.dsyrk
    assert f("X", "N", 2, 2, 1.0, a, 2, 0.0, b, 2, lib=lib) == 1
    assert f("L", "X", 2, 2, 1.0, a, 2, 0.0, b, 2, lib=lib) == 2
    assert f("L", "N", -1, 2, 1.0, a, 2, 0.0, b, 2, lib=lib) == 3
    assert f("L", "N", 2, -1, 1.0, a, 2, 0.0, b, 2, lib=lib) == 4
    assert f("L", "N", 2, 2, 1.0, None, 2, 0.0, b, 2, lib=lib) == 6
    assert f("L", "N", 4, 2, 1.0, a, 3, 0.0, b, 4, lib=lib) == 7          # lda < n for 'N'
    assert f("L", "T", 4, 2, 1.0, a, 2, 0.0, b, 4, lib=lib) == 0          # lda >= k for 'T'
    assert f("L", "T", 2, 4, 1.0, a, 3, 0.0, b, 2, lib=lib) == 7          # lda < k for 'T'
    assert f("L", "N", 2, 2, 1.0, a, 2, 0.0, None, 2, lib=lib) == 9
    assert f("L", "T", 4, 2, 1.0, a, 2, 0.0, b, 3, lib=lib) == 10         # ldc < n


ALL_PINS = [pin_blas3_library, pin_blas3_integer_exact, pin_blas3_closed_forms,
            pin_blas3_untouched, pin_blas3_zero_rules, pin_blas3_threads, pin_blas3_validation]

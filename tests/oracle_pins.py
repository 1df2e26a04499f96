"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each pin takes an oracle library handle (None = the built oracle) and raises
AssertionError on a mismatch. They are collected by test_oracle.py and re-run
against deliberately broken builds of the oracle by test_oracle_mutants.py,
which checks that every planted mistake trips at least one pin.

What pins what:
  golden_ld       the paper's leading-dimension example (section 1.2) and the
                  column-major map j*ld + i (section 2.3)
  ones            closed form: A = B = all ones gives C = alpha*k + beta*C0
  identity        closed form: A = I gives op(B), B = I gives op(A), bitwise
  permutation     closed form: permutation matrices move rows/columns, bitwise
  integer_exact   integer-valued inputs: every product and partial sum is an
                  exact binary64 value, so the result must equal exact integer
                  arithmetic (numpy int64 matmul as the library routine)
  rational        exact rational evaluation (fractions) of the same inputs;
                  the oracle is within the dot-product bound gamma_{k+2} * D
                  (Higham, Accuracy and Stability, section 3.1), and its
                  error denominator D equals the exact one to rounding
  library_matmul  alpha=1, beta=0, NN reduces to a plain matrix product:
                  numpy's matmul within 2*gamma_k*|A||B|
  transpose       C^T = op(B)^T op(A)^T: the transposed problem gives the
                  transposed result bitwise; stored transposes under 'T'
                  equal the originals under 'N' bitwise
  zero_rules      BLAS conventions: beta = 0 ignores C0; alpha = 0 or k = 0
                  never reads A, B; m = 0 or n = 0 touches nothing
  nan_row         a NaN in A(i,p) poisons row i of C and nothing else
  threads         bitwise independence of the OpenMP thread count
  validation      argument-check codes in argument order
  bruteforce      a pure-Python float loop on tiny shapes, bitwise
  dd_rational     the doubled-precision reference (oracle_dgemm_dd) against exact
                  rationals: within one rounding of the exact result plus
                  gamma_k^2 * D (Ogita, Rump and Oishi 2005, the Dot2 bound)
  dd_cancellation constructed cancellations where the plain loop returns 0 and
                  the exact answer is a product's or a sum's rounding error
                  (each error term of TwoProduct/TwoSum, and of alpha*s and
                  beta*c0, is the whole answer in one case)
  dd_integer      integer-valued inputs: the reference equals the plain loop
                  bitwise (both exact)
"""
from __future__ import annotations

import itertools
import os
from fractions import Fraction

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
U = 2.0 ** -53
TRANS = ("N", "T")


def _gamma(n: int) -> float:
    return n * U / (1 - n * U)


def _op(x, trans, rows_op, cols_op, ld):
    """op(X) as a dense 2-D numpy array (data movement only)."""
    r, c = synth.stored_dims(trans, rows_op, cols_op)
    v = synth.view2d(x, r, c, ld)
    return v.T if synth.is_trans(trans) else v


def _run(lib, p, alpha, beta, C=None):
    C = p["C"].copy() if C is None else C
    info = oracle.dgemm(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha,
                        p["A"], p["lda"], p["B"], p["ldb"], beta, C, p["ldc"], lib=lib)
    assert info == 0, f"oracle returned {info}"
    return C


def _pad3(rows):
    return max(1, rows) + 3


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def _same(x, y):
    """Bitwise equality except that -0 == +0 and NaN == NaN."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    both_nan = np.isnan(x) & np.isnan(y)
    return bool(np.all(both_nan | (x == y)))


def _pad_rows_untouched(p, C):
    m, n, ldc = p["m"], p["n"], p["ldc"]
    if ldc > m and n > 0:
        assert np.all(_bits(C).reshape(n, ldc)[:, m:] == synth.PAD_C_BITS), "C padding written"


SHAPES = [(1, 1, 1), (3, 5, 7), (16, 16, 16), (17, 15, 33), (33, 31, 13), (8, 40, 3)]


# ----------------------------------------------------------------------------
def pin_golden_ld(lib=None):
    path = os.path.join(HERE, "golden", "leading_dimension_example.txt")
    fields = {}
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "row":
            rows.append([float(v) for v in vals])
        else:
            fields[key] = vals
    store = np.array([float(v) for v in fields["storage"]])
    off, ld = int(fields["offset"][0]), int(fields["ld"][0])
    r, c = int(fields["rows"][0]), int(fields["cols"][0])
    sub = np.array(rows)
    A = store[off:].copy()  # the matrix passed by the address of its (0,0) entry
    eye = np.eye(c).T.reshape(-1).copy()
    for ta, expect in (("N", sub), ("T", sub.T)):
        C = np.full(r * c, np.nan)
        info = oracle.dgemm(ta, "N", r, c, c, 1.0, A, ld, eye, c, 0.0, C, r, lib=lib)
        assert info == 0
        got = C.reshape(c, r).T
        assert np.array_equal(got, expect), f"leading-dimension example, trans {ta}"


def pin_ones(lib=None):
    for (m, n, k), ta, tb in itertools.product(SHAPES + [(0, 3, 2), (5, 4, 0)], TRANS, TRANS):
        p = synth.problem(90, 0, ta, tb, m, n, k, ld_rule=_pad3, dist="ones", c_dist="int")
        C0 = p["C"].copy()
        C = _run(lib, p, 1.5, 0.5)
        got = synth.view2d(C, m, n, p["ldc"])
        want = 1.5 * k + 0.5 * synth.view2d(C0, m, n, p["ldc"])
        assert np.array_equal(got, want), f"all-ones closed form {ta}{tb} {m}x{n}x{k}"
        _pad_rows_untouched(p, C)


def pin_identity(lib=None):
    for (m, n, _), ta, tb in itertools.product(SHAPES, TRANS, TRANS):
        # A = I (k = m): C = op(B)
        p = synth.problem(91, 0, ta, tb, m, n, m, ld_rule=_pad3)
        a = synth.view2d(p["A"], m, m, p["lda"])
        a[:, :] = np.eye(m)
        C = _run(lib, p, 1.0, 0.0)
        want = _op(p["B"], tb, m, n, p["ldb"])
        assert _same(synth.view2d(C, m, n, p["ldc"]), want), f"A = I, {ta}{tb} {m}x{n}"
        # B = I (k = n): C = op(A)
        p = synth.problem(91, 1, ta, tb, m, n, n, ld_rule=_pad3)
        b = synth.view2d(p["B"], n, n, p["ldb"])
        b[:, :] = np.eye(n)
        C = _run(lib, p, 1.0, 0.0)
        want = _op(p["A"], ta, m, n, p["lda"])
        assert _same(synth.view2d(C, m, n, p["ldc"]), want), f"B = I, {ta}{tb} {m}x{n}"


def pin_permutation(lib=None):
    g = synth.rng(synth.seed_for(92, 0, 9))
    for (m, n, k), ta, tb in itertools.product(SHAPES, TRANS, TRANS):
        # op(A) = P (m x m permutation, P[i, s[i]] = 1): C[i, :] = op(B)[s[i], :]
        s = g.permutation(m)
        P = np.zeros((m, m))
        P[np.arange(m), s] = 1.0
        p = synth.problem(92, 1, ta, tb, m, n, m, ld_rule=_pad3)
        stored = synth.view2d(p["A"], m, m, p["lda"])
        stored[:, :] = P.T if synth.is_trans(ta) else P
        C = _run(lib, p, 1.0, 0.0)
        opb = _op(p["B"], tb, m, n, p["ldb"])
        assert _same(synth.view2d(C, m, n, p["ldc"]), opb[s, :]), f"row permutation {ta}{tb}"
        # op(B) = Q (n x n, Q[t[j], j] = 1): C[:, j] = op(A)[:, t[j]]
        t = g.permutation(n)
        Q = np.zeros((n, n))
        Q[t, np.arange(n)] = 1.0
        p = synth.problem(92, 2, ta, tb, m, n, n, ld_rule=_pad3)
        stored = synth.view2d(p["B"], n, n, p["ldb"])
        stored[:, :] = Q.T if synth.is_trans(tb) else Q
        C = _run(lib, p, 1.0, 0.0)
        opa = _op(p["A"], ta, m, n, p["lda"])
        assert _same(synth.view2d(C, m, n, p["ldc"]), opa[:, t]), f"column permutation {ta}{tb}"


def pin_integer_exact(lib=None):
    shapes = SHAPES + [(64, 64, 300), (70, 5, 129)]
    cases = [(1.5, 0.5), (2.0, -3.0), (-1.0, 0.0), (1.0, 1.0)]
    for (m, n, k), ta, tb in itertools.product(shapes, TRANS, TRANS):
        for v, (alpha, beta) in enumerate(cases):
            p = synth.problem(93, v, ta, tb, m, n, k, ld_rule=_pad3, dist="int")
            C0 = synth.view2d(p["C"], m, n, p["ldc"]).astype(np.int64)
            C = _run(lib, p, alpha, beta)
            ai = _op(p["A"], ta, m, k, p["lda"]).astype(np.int64)
            bi = _op(p["B"], tb, k, n, p["ldb"]).astype(np.int64)
            prod = ai @ bi
            # alpha, beta are multiples of 1/2: compare 2*C exactly in int64
            want2 = int(2 * alpha) * prod + (int(2 * beta) * C0 if beta != 0 else 0)
            got2 = 2 * synth.view2d(C, m, n, p["ldc"])
            assert np.array_equal(got2, want2.astype(np.float64)), \
                f"integer exactness {ta}{tb} {m}x{n}x{k} alpha={alpha} beta={beta}"
            _pad_rows_untouched(p, C)


def pin_rational(lib=None):
    shapes = [(1, 1, 1), (2, 3, 4), (4, 3, 9), (3, 2, 17)]
    for (m, n, k), ta, tb in itertools.product(shapes, TRANS, TRANS):
        alpha, beta = 0.7, -1.3
        p = synth.problem(94, 0, ta, tb, m, n, k, ld_rule=_pad3)
        C0 = synth.view2d(p["C"], m, n, p["ldc"]).copy()
        C = _run(lib, p, alpha, beta)
        D = np.zeros(m * n)
        info = oracle.absden(ta, tb, m, n, k, alpha, p["A"], p["lda"], p["B"], p["ldb"],
                             beta, p["C"], p["ldc"], D, m, lib=lib)
        assert info == 0
        D = D.reshape(n, m).T
        a = _op(p["A"], ta, m, k, p["lda"])
        b = _op(p["B"], tb, k, n, p["ldb"])
        got = synth.view2d(C, m, n, p["ldc"])
        for i in range(m):
            for j in range(n):
                s = sum(Fraction(a[i, q]) * Fraction(b[q, j]) for q in range(k))
                exact = Fraction(alpha) * s + Fraction(beta) * Fraction(C0[i, j])
                dex = abs(Fraction(alpha)) * sum(abs(Fraction(a[i, q]) * Fraction(b[q, j]))
                                                 for q in range(k)) \
                    + abs(Fraction(beta)) * abs(Fraction(C0[i, j]))
                err = abs(Fraction(got[i, j]) - exact)
                assert err <= Fraction(_gamma(k + 2)) * dex, f"rational bound {ta}{tb} ({i},{j})"
                assert abs(Fraction(D[i, j]) - dex) <= Fraction(_gamma(k + 2)) * dex, \
                    f"error denominator {ta}{tb} ({i},{j})"


def pin_library_matmul(lib=None):
    for (m, n, k) in [(40, 33, 50), (7, 64, 129)]:
        p = synth.problem(95, 0, "N", "N", m, n, k, ld_rule=_pad3)
        C = _run(lib, p, 1.0, 0.0)
        a = _op(p["A"], "N", m, k, p["lda"])
        b = _op(p["B"], "N", k, n, p["ldb"])
        ref = a @ b
        bound = 2 * _gamma(k) * (np.abs(a) @ np.abs(b))
        assert np.all(np.abs(synth.view2d(C, m, n, p["ldc"]) - ref) <= bound), "numpy matmul"


def pin_transpose(lib=None):
    for (m, n, k) in SHAPES:
        alpha, beta = 1.25, -0.75
        p = synth.problem(96, 0, "N", "N", m, n, k, ld_rule=_pad3)
        Cn = _run(lib, p, alpha, beta)
        # transposed problem: C^T (n x m) = alpha * B^T A^T + beta * C0^T
        c0t = np.ascontiguousarray(synth.view2d(p["C"], m, n, p["ldc"]).T)
        ct = c0t.T.reshape(-1).copy()  # flat column-major storage of C0^T, ld = n
        info = oracle.dgemm("T", "T", n, m, k, alpha, p["B"], p["ldb"], p["A"], p["lda"],
                            beta, ct, n, lib=lib)
        assert info == 0
        assert _same(ct.reshape(m, n), synth.view2d(Cn, m, n, p["ldc"])), f"(AB)^T = B^T A^T {m}x{n}x{k}"
        # materialised transposes under 'T' equal the originals under 'N'
        a = _op(p["A"], "N", m, k, p["lda"])
        b = _op(p["B"], "N", k, n, p["ldb"])
        # row-major a (m x k) is the column-major storage of A^T (k x m, ld = k);
        # likewise row-major b is the storage of B^T (n x k, ld = n)
        at = np.ascontiguousarray(a).reshape(-1)
        bt = np.ascontiguousarray(b).reshape(-1)
        C2 = p["C"].copy()
        info = oracle.dgemm("T", "T", m, n, k, alpha, at, max(1, k), bt, max(1, n),
                            beta, C2, p["ldc"], lib=lib)
        assert info == 0
        assert _same(C2, Cn), f"stored transposes {m}x{n}x{k}"


def pin_zero_rules(lib=None):
    m, n, k = 7, 5, 6
    p = synth.problem(97, 0, "N", "N", m, n, k, ld_rule=_pad3)
    nanC = p["C"].copy()
    synth.view2d(nanC, m, n, p["ldc"])[:, :] = np.nan
    # beta == 0: C0 is not read
    C = _run(lib, p, 1.0, 0.0, C=nanC.copy())
    assert np.all(np.isfinite(synth.view2d(C, m, n, p["ldc"]))), "beta=0 read C0"
    # alpha == 0: A and B are not read (NULL is accepted) and C := beta*C0
    for beta in (0.0, 2.0):
        C = p["C"].copy()
        info = oracle.dgemm("N", "N", m, n, k, 0.0, None, p["lda"], None, p["ldb"], beta, C,
                            p["ldc"], lib=lib)
        assert info == 0
        want = 0.0 * synth.view2d(p["C"], m, n, p["ldc"]) if beta == 0 else \
            beta * synth.view2d(p["C"], m, n, p["ldc"])
        assert np.array_equal(synth.view2d(C, m, n, p["ldc"]), want), "alpha=0 rule"
        _pad_rows_untouched(p, C)
    # beta == 0 and alpha == 0 with C0 = NaN: exact zeros
    C = nanC.copy()
    assert oracle.dgemm("N", "N", m, n, k, 0.0, None, p["lda"], None, p["ldb"], 0.0, C,
                        p["ldc"], lib=lib) == 0
    assert np.all(synth.view2d(C, m, n, p["ldc"]) == 0.0), "alpha=beta=0 must give zeros"
    # k == 0: C := beta*C0
    C = p["C"].copy()
    assert oracle.dgemm("N", "N", m, n, 0, 1.0, None, max(1, m), None, 1, 3.0, C, p["ldc"],
                        lib=lib) == 0
    assert np.array_equal(synth.view2d(C, m, n, p["ldc"]), 3.0 * synth.view2d(p["C"], m, n, p["ldc"]))
    # quick return: (alpha == 0 or k == 0) and beta == 1 leaves C bitwise alone (NaN too)
    C = nanC.copy()
    assert oracle.dgemm("N", "N", m, n, k, 0.0, None, p["lda"], None, p["ldb"], 1.0, C,
                        p["ldc"], lib=lib) == 0
    assert np.array_equal(_bits(C), _bits(nanC)), "quick return touched C"
    # m == 0 or n == 0: nothing is touched, even through NULL pointers
    assert oracle.dgemm("N", "N", 0, n, k, 1.0, None, 1, None, k, 0.0, None, 1, lib=lib) == 0
    assert oracle.dgemm("N", "N", m, 0, k, 1.0, None, m, None, k, 0.0, None, m, lib=lib) == 0


def pin_nan_row(lib=None):
    m, n, k = 9, 8, 10
    for ta, tb in itertools.product(TRANS, TRANS):
        p = synth.problem(98, 0, ta, tb, m, n, k, ld_rule=_pad3)
        i0, p0 = 4, 7
        r, c = synth.stored_dims(ta, m, k)
        st = synth.view2d(p["A"], r, c, p["lda"])
        if synth.is_trans(ta):
            st[p0, i0] = np.nan
        else:
            st[i0, p0] = np.nan
        C = _run(lib, p, 1.0, 0.5)
        nan = np.isnan(synth.view2d(C, m, n, p["ldc"]))
        want = np.zeros((m, n), dtype=bool)
        want[i0, :] = True
        assert np.array_equal(nan, want), f"NaN in A({i0},{p0}) must poison row {i0} only ({ta}{tb})"


def pin_threads(lib=None):
    p = synth.problem(99, 0, "T", "N", 61, 47, 83, ld_rule=_pad3)
    before = oracle.get_threads(lib=lib)
    try:
        oracle.set_threads(1, lib=lib)
        c1 = _run(lib, p, 0.9, 1.1)
        oracle.set_threads(8, lib=lib)
        c8 = _run(lib, p, 0.9, 1.1)
    finally:
        oracle.set_threads(before, lib=lib)
    assert np.array_equal(_bits(c1), _bits(c8)), "thread-count dependence"


def pin_validation(lib=None):
    a = np.zeros(64)
    b = np.zeros(64)
    c = np.zeros(64)

    def call(ta="N", tb="N", m=4, n=4, k=4, lda=4, ldb=4, ldc=4, A=a, B=b, C=c, alpha=1.0):
        return oracle.dgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, 0.0, C, ldc, lib=lib)

    assert call() == 0
    assert call(ta="n", tb="t") == 0 and call(ta="C", tb="c") == 0
    assert call(ta="X") == 1
    assert call(tb="x") == 2
    assert call(m=-1) == 3
    assert call(n=-1) == 4
    assert call(k=-1) == 5
    assert call(A=None) == 7
    assert call(lda=3) == 8
    assert call(ta="T", m=8, k=4, lda=4, ldc=8) == 0  # stored A is k x m: lda >= k
    assert call(ta="T", m=4, k=8, lda=4) == 8
    assert call(B=None) == 9
    assert call(ldb=3) == 10
    assert call(tb="T", n=8, k=4, ldb=4) == 10  # stored B is n x k: ldb >= n
    assert call(C=None) == 12
    assert call(ldc=3) == 13
    assert call(m=0, lda=1, ldc=1) == 0
    assert call(m=0, lda=0) == 8  # ld >= 1 even for empty matrices
    assert call(ta="X", m=-1) == 1  # first bad argument wins


def _py_dgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    for j in range(n):
        for i in range(m):
            s = 0.0
            for q in range(k):
                a = A[i * lda + q] if ta == "T" else A[q * lda + i]
                b = B[q * ldb + j] if tb == "T" else B[j * ldb + q]
                s = s + float(a) * float(b)
            C[j * ldc + i] = alpha * s if beta == 0 else alpha * s + beta * float(C[j * ldc + i])


def pin_bruteforce(lib=None):
    dims = (0, 1, 2, 3, 5, 8)
    ab = [(1.0, 0.0), (1.5, 0.5), (-1.0, 1.0), (0.3, -2.7)]
    g = synth.rng(synth.seed_for(100, 0, 9))
    for m, n, k in itertools.product(dims, dims, (1, 3, 8)):
        ta, tb = TRANS[int(g.integers(2))], TRANS[int(g.integers(2))]
        alpha, beta = ab[int(g.integers(len(ab)))]
        p = synth.problem(100, 1, ta, tb, m, n, k, ld_rule=_pad3)
        C = _run(lib, p, alpha, beta)
        ref = p["C"].copy()
        _py_dgemm(ta, tb, m, n, k, alpha, p["A"], p["lda"], p["B"], p["ldb"], beta, ref, p["ldc"])
        assert np.array_equal(_bits(C), _bits(ref)), f"pure-Python loop {ta}{tb} {m}x{n}x{k}"


def _run_dd(lib, p, alpha, beta, C=None):
    C = p["C"].copy() if C is None else C
    info = oracle.dgemm_dd(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha,
                           p["A"], p["lda"], p["B"], p["ldb"], beta, C, p["ldc"], lib=lib)
    assert info == 0, f"oracle_dgemm_dd returned {info}"
    return C


def pin_dd_rational(lib=None):
    shapes = [(1, 1, 1), (2, 3, 4), (4, 3, 9), (3, 2, 17)]
    for (m, n, k), ta, tb in itertools.product(shapes, TRANS, TRANS):
        alpha, beta = 0.7, -1.3
        p = synth.problem(95, 0, ta, tb, m, n, k, ld_rule=_pad3)
        C0 = synth.view2d(p["C"], m, n, p["ldc"]).copy()
        got = synth.view2d(_run_dd(lib, p, alpha, beta), m, n, p["ldc"])
        a = _op(p["A"], ta, m, k, p["lda"])
        b = _op(p["B"], tb, k, n, p["ldb"])
        for i in range(m):
            for j in range(n):
                s = sum(Fraction(a[i, q]) * Fraction(b[q, j]) for q in range(k))
                exact = Fraction(alpha) * s + Fraction(beta) * Fraction(C0[i, j])
                dex = abs(Fraction(alpha)) * sum(abs(Fraction(a[i, q]) * Fraction(b[q, j]))
                                                 for q in range(k)) \
                    + abs(Fraction(beta)) * abs(Fraction(C0[i, j]))
                bound = Fraction(2 * U) * abs(exact) + Fraction(4 * _gamma(k + 2) ** 2) * dex
                assert abs(Fraction(got[i, j]) - exact) <= bound, f"dd rational {ta}{tb} ({i},{j})"


def _dot_case(lib, x, y, alpha=1.0, beta=0.0, c0=0.0):
    """alpha * x'y + beta * c0 through the reference (m = n = 1, op = N)."""
    k = len(x)
    C = np.array([c0], dtype=np.float64)
    info = oracle.dgemm_dd("N", "N", 1, 1, k, alpha, np.array(x, dtype=np.float64), 1,
                           np.array(y, dtype=np.float64), max(1, k), beta, C, 1, lib=lib)
    assert info == 0
    return C[0]


def pin_dd_cancellation(lib=None):
    e = 2.0 ** -30
    a = 1.0 + e                      # a * a = 1 + 2^-29 + 2^-60: its rounding error is 2^-60
    aa = a * a                       # binary64 product (1 + 2^-29)
    assert float(Fraction(a) * Fraction(a) - Fraction(aa)) == 2.0 ** -60
    # a sum's rounding error is the answer: 2^60 + 1.5 rounds to 2^60
    assert _dot_case(lib, [2.0 ** 60, 1.5, -(2.0 ** 60)], [1.0, 1.0, 1.0]) == 1.5, "TwoSum error"
    # a product's rounding error is the answer: a*a - fl(a*a)
    assert _dot_case(lib, [a, -1.0], [a, aa]) == 2.0 ** -60, "TwoProduct error"
    # alpha * s has a rounding error that beta * c0 cancels down to
    assert _dot_case(lib, [a], [1.0], alpha=a, beta=-1.0, c0=aa) == 2.0 ** -60, "alpha*s error"
    # beta * c0 has the rounding error
    assert _dot_case(lib, [aa], [1.0], alpha=-1.0, beta=a, c0=a) == 2.0 ** -60, "beta*c0 error"
    # and the plain loop indeed returns 0 on the first two (what the reference is for)
    C = np.array([0.0])
    oracle.dgemm("N", "N", 1, 1, 3, 1.0, np.array([2.0 ** 60, 1.5, -(2.0 ** 60)]), 1,
                 np.ones(3), 3, 0.0, C, 1, lib=lib)
    assert C[0] == 0.0


def pin_dd_integer(lib=None):
    for ta, tb in itertools.product(TRANS, TRANS):
        p = synth.problem(96, 0, ta, tb, 13, 11, 29, ld_rule=_pad3, dist="int")
        plain = _run(lib, p, 1.5, 0.5)
        dd = _run_dd(lib, p, 1.5, 0.5)
        assert np.array_equal(_bits(plain), _bits(dd)), f"dd integer {ta}{tb}"
        _pad_rows_untouched(p, dd)


ALL_PINS = [pin_golden_ld, pin_ones, pin_identity, pin_permutation, pin_integer_exact,
            pin_rational, pin_library_matmul, pin_transpose, pin_zero_rules, pin_nan_row,
            pin_threads, pin_validation, pin_bruteforce, pin_dd_rational, pin_dd_cancellation,
            pin_dd_integer]

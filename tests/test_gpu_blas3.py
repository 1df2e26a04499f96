"""GPU parity of the level-3 operations built on the GEMM (mdg_dsyrk, mdg_dtrmm, mdg_dtrsm)
against the CPU oracle (oracle_dsyrk, oracle_dtrmm, oracle_dtrsm, pinned in blas3_pins.py).

Integer-valued data: every sum is exact in any order, so results equal the oracle exactly (for
the solve, B is built as 2 op(A) X0 by the oracle's multiply with integer X0 and powers of two on
the diagonal, so the solution is X0). Uniform data: syrk and trmm within 1e-13 D with
D = |alpha| |op(A)| |op(B)| (+ |beta| |C0|), as for the GEMM; trsm by its residual
alpha B - op(A) X (or alpha B - X op(A)) evaluated in doubled precision by the oracle, within
1e-13 (|op(A)| |X| + |alpha| |B|), and within 1e-12 max|X| of the oracle's substitution.
Orders cross the 64-row leaf of the triangular recursion several times (up to four levels of
halving) and end in ragged blocks; the triangle not named by uplo, a unit diagonal and all padding
hold NaN.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, sample_indices, to_dev

pytestmark = pytest.mark.gpu

COMBOS = list(itertools.product("LR", "LU", "NT", "NU"))
TRI_SHAPES = [(1, 1), (7, 5), (64, 64), (65, 33), (130, 70), (200, 300), (700, 90), (90, 1100)]
SYRK_SHAPES = [(1, 1), (5, 3), (64, 16), (65, 17), (130, 70), (257, 129), (300, 513)]


def _mdg():
    import paper_1609_00076_amd as mdg
    return mdg


def _sync_host(d):
    import torch
    torch.cuda.synchronize()
    return d.cpu().numpy()


def _dense_op(Aflat, na, lda, uplo, transa, diag):
    """op(A) of a stored triangular A as a dense array (zeros off the triangle, ones on a unit
    diagonal): the denominators' |op(A)| and the residual's operand."""
    S = synth.view2d(Aflat, na, na, lda).copy()
    S[np.isnan(S)] = 0.0
    T = np.tril(S) if uplo == "L" else np.triu(S)
    if diag == "U":
        np.fill_diagonal(T, 1.0)
    return T.T.copy() if transa == "T" else T


def _tri_case(seed, side, uplo, transa, diag, m, n, dist):
    na = m if side == "L" else n
    lda, ldb = na + 3, m + 2
    A = synth.triangular(synth.seed_for(60, seed, 0), na, lda, uplo, "int" if dist == "int" else
                         "uniform", unit=(diag == "U"))
    B = synth.matrix(synth.seed_for(60, seed, 1), m, n, ldb, "int" if dist == "int" else "uniform")
    return na, A, lda, B, ldb


def _run_tri(name, side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb):
    mdg = _mdg()
    dA, dB = to_dev(A), to_dev(B)
    st = getattr(mdg, name)(side, uplo, transa, diag, m, n, alpha, dA, lda, dB, ldb)
    assert st == 0, (name, st, mdg.mdg_status_string(st))
    return _sync_host(dB)


def _pad_same(got, ref, rows, ld):
    """The padding rows of two flat column-major arrays are bitwise equal."""
    cols = got.size // ld
    g = got.reshape(cols, ld)[:, rows:].view(np.uint64)
    r = ref.reshape(cols, ld)[:, rows:].view(np.uint64)
    return np.array_equal(g, r)


@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(c))
@pytest.mark.parametrize("shape", TRI_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_trmm_integer_exact(combo, shape):
    side, uplo, transa, diag = combo
    m, n = shape
    na, A, lda, B, ldb = _tri_case(1, side, uplo, transa, diag, m, n, "int")
    ref = B.copy()
    assert oracle.dtrmm(side, uplo, transa, diag, m, n, 2.0, A, lda, ref, ldb) == 0
    got = _run_tri("mdg_dtrmm", side, uplo, transa, diag, m, n, 2.0, A, lda, B, ldb)
    assert np.array_equal(synth.view2d(got, m, n, ldb), synth.view2d(ref, m, n, ldb))
    assert _pad_same(got, B, m, ldb)


@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(c))
@pytest.mark.parametrize("shape", TRI_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_trmm_uniform(combo, shape):
    side, uplo, transa, diag = combo
    m, n = shape
    na, A, lda, B, ldb = _tri_case(2, side, uplo, transa, diag, m, n, "uniform")
    alpha = -0.75
    ref = B.copy()
    assert oracle.dtrmm(side, uplo, transa, diag, m, n, alpha, A, lda, ref, ldb) == 0
    got = _run_tri("mdg_dtrmm", side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb)
    T = np.abs(_dense_op(A, na, lda, uplo, transa, diag))
    Bl = np.abs(synth.view2d(B, m, n, ldb))
    D = abs(alpha) * (T @ Bl if side == "L" else Bl @ T)
    err = np.abs(synth.view2d(got, m, n, ldb) - synth.view2d(ref, m, n, ldb))
    assert np.all(err <= TOL * D), float(np.max(err / np.maximum(D, 1e-300)))
    assert _pad_same(got, B, m, ldb)


@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(c))
def test_trmm_nonfinite_entries(combo):
    """An infinity and a NaN in B reach exactly the entries the oracle's triangle loops give them
    to (integer data, so every finite entry is exact as well)."""
    side, uplo, transa, diag = combo
    m, n = 130, 70
    na, A, lda, B, ldb = _tri_case(5, side, uplo, transa, diag, m, n, "int")
    Bl = synth.view2d(B, m, n, ldb)
    Bl[3, 5] = np.inf
    Bl[100, 60] = -np.inf
    Bl[70, 2] = np.nan
    ref = B.copy()
    assert oracle.dtrmm(side, uplo, transa, diag, m, n, 2.0, A, lda, ref, ldb) == 0
    got = _run_tri("mdg_dtrmm", side, uplo, transa, diag, m, n, 2.0, A, lda, B, ldb)
    g, r = synth.view2d(got, m, n, ldb), synth.view2d(ref, m, n, ldb)
    assert np.array_equal(g, r, equal_nan=True)
    assert np.isfinite(r).sum() > m * n // 2  # most entries stay finite


@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(c))
@pytest.mark.parametrize("shape", TRI_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_trsm_integer_exact(combo, shape):
    side, uplo, transa, diag = combo
    m, n = shape
    na, A, lda, X0, ldb = _tri_case(3, side, uplo, transa, diag, m, n, "int")
    B = X0.copy()
    assert oracle.dtrmm(side, uplo, transa, diag, m, n, 2.0, A, lda, B, ldb) == 0  # B = 2 op(A) X0
    ref = B.copy()
    assert oracle.dtrsm(side, uplo, transa, diag, m, n, 0.5, A, lda, ref, ldb) == 0
    got = _run_tri("mdg_dtrsm", side, uplo, transa, diag, m, n, 0.5, A, lda, B, ldb)
    want = synth.view2d(X0, m, n, ldb)
    assert np.array_equal(synth.view2d(ref, m, n, ldb), want)  # the oracle recovers X0
    assert np.array_equal(synth.view2d(got, m, n, ldb), want)
    assert _pad_same(got, B, m, ldb)


def _residual_check(side, m, n, alpha, T, B0, ldb, X):
    """max |alpha B0 - op(A) X| / (|op(A)||X| + |alpha||B0|) with the residual from the oracle's
    doubled-precision GEMM (the triangle as a dense operand)."""
    Xl = np.asfortranarray(synth.view2d(X, m, n, ldb))
    Bl = synth.view2d(B0, m, n, ldb)
    R = np.asfortranarray(Bl).ravel(order="F").copy()
    Tf = np.asfortranarray(T).ravel(order="F").copy()
    Xf = Xl.ravel(order="F").copy()
    na = T.shape[0]
    if side == "L":
        assert oracle.dgemm_dd("N", "N", m, n, na, -1.0, Tf, na, Xf, m, alpha, R, m) == 0
        D = np.abs(T) @ np.abs(Xl) + abs(alpha) * np.abs(Bl)
    else:
        assert oracle.dgemm_dd("N", "N", m, n, na, -1.0, Xf, m, Tf, na, alpha, R, m) == 0
        D = np.abs(Xl) @ np.abs(T) + abs(alpha) * np.abs(Bl)
    R = R.reshape(n, m).T
    return float(np.max(np.abs(R) / D))


@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(c))
@pytest.mark.parametrize("shape", TRI_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_trsm_uniform(combo, shape):
    side, uplo, transa, diag = combo
    m, n = shape
    na, A, lda, B, ldb = _tri_case(4, side, uplo, transa, diag, m, n, "uniform")
    alpha = 1.5
    ref = B.copy()
    assert oracle.dtrsm(side, uplo, transa, diag, m, n, alpha, A, lda, ref, ldb) == 0
    got = _run_tri("mdg_dtrsm", side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb)
    T = _dense_op(A, na, lda, uplo, transa, diag)
    assert _residual_check(side, m, n, alpha, T, B, ldb, got) <= TOL
    g, r = synth.view2d(got, m, n, ldb), synth.view2d(ref, m, n, ldb)
    assert np.max(np.abs(g - r)) <= 1e-12 * np.max(np.abs(r))
    assert _pad_same(got, B, m, ldb)


@pytest.mark.parametrize("name", ["mdg_dtrmm", "mdg_dtrsm"])
def test_tri_alpha_zero_and_empty(name):
    mdg = _mdg()
    import torch
    m, n = 70, 9
    dB = torch.full((m * n,), float("nan"), dtype=torch.float64, device="cuda")
    st = getattr(mdg, name)("L", "L", "N", "N", m, n, 0.0, None, m, dB, m)
    assert st == 0
    assert np.array_equal(_sync_host(dB), np.zeros(m * n))
    dB = torch.full((4,), 3.0, dtype=torch.float64, device="cuda")
    assert getattr(mdg, name)("R", "U", "T", "U", 0, 4, 1.0, None, 4, dB, 1) == 0
    assert np.array_equal(_sync_host(dB), np.full(4, 3.0))
    d16 = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert getattr(mdg, name)("X", "U", "T", "U", 4, 4, 1.0, d16, 4, d16, 4) == 1
    assert getattr(mdg, name)("L", "U", "T", "U", 4, 4, 1.0, d16, 3, d16, 4) == 9


def _syrk_case(seed, uplo, trans, n, k, dist):
    ra, ca = (n, k) if trans == "N" else (k, n)
    lda, ldc = ra + 1, n + 3
    A = synth.matrix(synth.seed_for(61, seed, 0), ra, ca, lda, dist)
    C = synth.matrix(synth.seed_for(61, seed, 2), n, n, ldc, dist, pad=synth.pad_c_value())
    other = np.triu(np.ones((n, n), bool), 1) if uplo == "L" else np.tril(np.ones((n, n), bool), -1)
    synth.view2d(C, n, n, ldc)[other] = synth.pad_c_value()  # never read or written
    return A, lda, C, ldc, other


def _run_syrk(variant, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    mdg = _mdg()
    dA, dC = (None if A is None else to_dev(A)), to_dev(C)
    st = mdg.mdg_dsyrk_ex(variant, uplo, trans, n, k, alpha, dA, lda, beta, dC, ldc)
    return st, _sync_host(dC)


def _syrk_accepts(variant, uplo):
    mdg = _mdg()
    # An accepted configuration returns 0 on a product that nothing needs (n == 0 returns early,
    # so probe with a real but tiny problem on the host-side checks only: alpha == 0, beta == 1).
    import torch
    dC = torch.zeros(1, dtype=torch.float64, device="cuda")
    return mdg.mdg_dsyrk_ex(variant, uplo, "N", 1, 1, 0.0, None, 1, 0.5, dC, 1) == 0


@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NT")
@pytest.mark.parametrize("shape", SYRK_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_syrk_every_variant(uplo, trans, shape):
    n, k = shape
    mdg = _mdg()
    accepted = [v for v in [-1] + list(range(mdg.mdg_num_variants())) if _syrk_accepts(v, uplo)]
    names = {mdg.mdg_variant_name(v) for v in accepted if v >= 0}
    assert len(names) == 5, names
    base = 100 * SYRK_SHAPES.index(shape) + 10 * "LU".index(uplo) + 4 * "NT".index(trans)
    for case, (dist, alpha, beta) in enumerate((("int", 1.5, -0.5), ("uniform", -1.25, 0.75),
                                                ("uniform", 1.0, 0.0))):
        A, lda, C, ldc, other = _syrk_case(base + case, uplo, trans, n, k, dist)
        if beta == 0.0:  # C is not read: NaN in the triangle must not matter
            tri = ~other
            synth.view2d(C, n, n, ldc)[tri] = np.nan
        ref = C.copy()
        assert oracle.dsyrk(uplo, trans, n, k, alpha, A, lda, beta, ref, ldc) == 0
        ra, ca = (n, k) if trans == "N" else (k, n)
        opA = synth.view2d(A, ra, ca, lda)
        opA = opA if trans == "N" else opA.T
        C0 = synth.view2d(C, n, n, ldc)
        D = abs(alpha) * (np.abs(opA) @ np.abs(opA).T)
        if beta != 0.0:
            D = D + abs(beta) * np.abs(np.where(other, 0.0, C0))
        for v in accepted:
            st, got = _run_syrk(v, uplo, trans, n, k, alpha, A, lda, beta, C, ldc)
            assert st == 0, (v, st)
            g, r = synth.view2d(got, n, n, ldc), synth.view2d(ref, n, n, ldc)
            assert np.array_equal(g[other].view(np.uint64), C0[other].view(np.uint64)), \
                f"variant {v}: other triangle touched"
            assert _pad_same(got, C, n, ldc), f"variant {v}: padding touched"
            tri = ~other
            if dist == "int":
                assert np.array_equal(g[tri], r[tri]), f"variant {v} ({mdg.mdg_variant_name(v)})"
            else:
                err = np.abs(g[tri] - r[tri])
                assert np.all(err <= TOL * D[tri]), (v, float(np.max(err / np.maximum(D[tri], 1e-300))))


@pytest.mark.parametrize("uplo", "LU")
def test_syrk_no_product_and_refusals(uplo):
    mdg = _mdg()
    n = 77
    A, lda, C, ldc, other = _syrk_case(5, uplo, "N", n, 4, "uniform")
    C0 = synth.view2d(C, n, n, ldc)
    for alpha, k, beta in ((0.0, 4, 2.0), (1.0, 0, -0.5), (0.0, 4, 0.0)):
        st, got = _run_syrk(-1, uplo, "N", n, k, alpha, A if alpha else None, lda, beta, C, ldc)
        assert st == 0
        g = synth.view2d(got, n, n, ldc)
        want = np.zeros_like(C0) if beta == 0.0 else beta * np.where(other, 0.0, C0)
        assert np.array_equal(g[~other], want[~other])
        assert np.array_equal(g[other].view(np.uint64), C0[other].view(np.uint64))
    st, got = _run_syrk(-1, uplo, "N", n, 4, 0.0, None, lda, 1.0, C, ldc)
    assert st == 0 and np.array_equal(got.view(np.uint64), C.view(np.uint64))
    # A GEMM variant without a ring configuration for the update is refused.
    names = [mdg.mdg_variant_name(v) for v in range(mdg.mdg_num_variants())]
    plain = names.index("mfma_f64_64x64x16_w32x32")
    st, _ = _run_syrk(plain, uplo, "N", n, 4, 1.0, A, lda, 0.5, C, ldc)
    assert st == -2  # MDG_ERR_VARIANT
    assert mdg.mdg_dsyrk("X", "N", n, 4, 1.0, None, lda, 0.5, None, ldc) == 1
    assert mdg.mdg_dsyrk(uplo, "N", n, 4, 1.0, None, n - 1, 0.5, None, ldc) == 6
    assert mdg.mdg_dsyrk(uplo, "T", n, 4, 1.0, to_dev(A), 3, 0.5, None, ldc) == 7


@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NT")
def test_syrk_split_against_oracle(uplo, trans):
    """n = 4096, k = 2048 with the automatic choice: the rectangles between diagonal blocks of
    order 1024 as GEMMs (one 2048^2, two 1024^2), then one launch over the four diagonal blocks;
    exact on integer data, within 1e-13 of |alpha| |op(A)||op(A)^T| + |beta||C| on uniform data
    (one flag case), the other triangle and the padding untouched."""
    n, k = 4096, 2048
    base = 700 + 10 * "LU".index(uplo) + 4 * "NT".index(trans)
    cases = [("int", 1.5, -0.5)] + ([("uniform", -1.25, 0.75)] if uplo + trans == "LN" else [])
    for case, (dist, alpha, beta) in enumerate(cases):
        A, lda, C, ldc, other = _syrk_case(base + case, uplo, trans, n, k, dist)
        ref = C.copy()
        assert oracle.dsyrk(uplo, trans, n, k, alpha, A, lda, beta, ref, ldc) == 0
        print(f"[syrk split] {uplo}{trans} {dist}", flush=True)
        st, got = _run_syrk(-1, uplo, trans, n, k, alpha, A, lda, beta, C, ldc)
        assert st == 0
        g, r = synth.view2d(got, n, n, ldc), synth.view2d(ref, n, n, ldc)
        C0 = synth.view2d(C, n, n, ldc)
        assert np.array_equal(g[other].view(np.uint64), C0[other].view(np.uint64))
        assert _pad_same(got, C, n, ldc)
        tri = ~other
        if dist == "int":
            assert np.array_equal(g[tri], r[tri])
        else:
            ra, ca = (n, k) if trans == "N" else (k, n)
            opA = synth.view2d(A, ra, ca, lda)
            opA = opA if trans == "N" else opA.T
            D = abs(alpha) * (np.abs(opA) @ np.abs(opA).T) + abs(beta) * np.abs(np.where(other, 0.0, C0))
            err = np.abs(g[tri] - r[tri])
            assert np.all(err <= TOL * D[tri]), float(np.max(err / np.maximum(D[tri], 1e-300)))


# ---- full size: the benchmark's shapes and launch configuration, checked on samples ---------------

BIG = 8192


def test_syrk_full_size_sampled():
    """n = k = 8192, lower, trans 'N' (the benchmark case): sampled columns of the triangle
    against the oracle's GEMM of the same columns (op(A) times the sampled rows of op(A))."""
    n = k = BIG
    lda, ldc = n, n
    A = synth.matrix(synth.seed_for(62, 0, 0), n, k, lda, "uniform")
    C = synth.matrix(synth.seed_for(62, 0, 2), n, n, ldc, "uniform")
    alpha, beta = 1.0, 1.0
    st, got = _run_syrk(-1, "L", "N", n, k, alpha, A, lda, beta, C, ldc)
    assert st == 0
    cols = sample_indices(n, 6, 62)
    Al = synth.view2d(A, n, k, lda)
    for j in cols:
        rows = np.arange(j, n)
        Ar = np.ascontiguousarray(Al[rows]).ravel()            # op(A)(rows, :)^T stored k x len
        aj = np.ascontiguousarray(Al[j]).copy()                 # op(A)(j, :)
        ref = C.reshape(n, ldc)[j, rows].copy()
        assert oracle.dgemm("T", "N", len(rows), 1, k, alpha, Ar, k, aj, k, beta, ref,
                            len(rows)) == 0
        D = np.abs(Al[rows]) @ np.abs(Al[j]) + np.abs(C.reshape(n, ldc)[j, rows])
        err = np.abs(got.reshape(n, ldc)[j, rows] - ref)
        assert np.all(err <= TOL * D), (j, float(np.max(err / D)))
        assert np.array_equal(got.reshape(n, ldc)[j, :j].view(np.uint64),
                              C.reshape(n, ldc)[j, :j].view(np.uint64))


@pytest.mark.parametrize("name", ["mdg_dtrmm", "mdg_dtrsm"])
def test_tri_full_size_sampled(name):
    """m = n = 8192, side 'L', lower, 'N', non-unit (the benchmark case): sampled columns of B,
    each an independent right-hand side, against the oracle on those columns (trmm) or by the
    doubled-precision residual (trsm)."""
    m = n = BIG
    A = synth.triangular(synth.seed_for(63, 0, 0), m, m, "L", "uniform")
    B = synth.matrix(synth.seed_for(63, 0, 1), m, n, m, "uniform")
    alpha = 1.0
    got = _run_tri(name, "L", "L", "N", "N", m, n, alpha, A, m, B, m)
    cols = sample_indices(n, 4, 63)
    Bs = np.ascontiguousarray(synth.view2d(B, m, n, m)[:, cols].T).ravel()
    Gs = np.ascontiguousarray(synth.view2d(got, m, n, m)[:, cols].T).ravel()
    if name == "mdg_dtrmm":
        ref = Bs.copy()
        assert oracle.dtrmm("L", "L", "N", "N", m, len(cols), alpha, A, m, ref, m) == 0
        T = np.abs(_dense_op(A, m, m, "L", "N", "N"))
        D = T @ np.abs(synth.view2d(Bs, m, len(cols), m))
        err = np.abs(synth.view2d(Gs, m, len(cols), m) - synth.view2d(ref, m, len(cols), m))
        assert np.all(err <= TOL * D)
    else:
        T = _dense_op(A, m, m, "L", "N", "N")
        assert _residual_check("L", m, len(cols), alpha, T, Bs, m, Gs) <= TOL


def test_level3_graph_replay_matches_eager():
    """dsyrk, dtrmm and dtrsm (about two hundred launches each at this size) captured in one
    graph on torch's stream: every replay, with eager work and synchronizations between replays,
    gives the eager results bit for bit."""
    import torch
    mdg = _mdg()
    n, k, m = 700, 300, 500
    hA = synth.matrix(synth.seed_for(65, 0, 0), n, k, n, "uniform")
    hC = synth.matrix(synth.seed_for(65, 0, 2), n, n, n, "uniform")
    hT = synth.triangular(synth.seed_for(65, 0, 3), m, m, "U", "uniform")
    hB = synth.matrix(synth.seed_for(65, 0, 1), m, n, m, "uniform")
    dA, dC0, dT, dB0 = (to_dev(x) for x in (hA, hC, hT, hB))
    dC, dB1, dB2 = dC0.clone(), dB0.clone(), dB0.clone()

    def calls():
        assert mdg.mdg_dsyrk("U", "N", n, k, 0.5, dA, n, 1.5, dC, n) == 0
        assert mdg.mdg_dtrmm("L", "U", "N", "N", m, n, 1.25, dT, m, dB1, m) == 0
        assert mdg.mdg_dtrsm("L", "U", "T", "U", m, n, -0.5, dT, m, dB2, m) == 0

    calls()  # eager results (also warms the library's per-device state)
    torch.cuda.synchronize()
    want = [x.clone() for x in (dC, dB1, dB2)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # torch's warm-up-before-capture on a side stream
        for x, x0 in ((dC, dC0), (dB1, dB0), (dB2, dB0)):
            x.copy_(x0)
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    for x, x0 in ((dC, dC0), (dB1, dB0), (dB2, dB0)):
        x.copy_(x0)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        calls()
    for rep in range(3):
        for x, x0 in ((dC, dC0), (dB1, dB0), (dB2, dB0)):
            x.copy_(x0)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for got, ref in zip((dC, dB1, dB2), want):
            assert torch.equal(got.view(torch.int64), ref.view(torch.int64)), f"replay {rep}"

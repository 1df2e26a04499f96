"""GPU parity of the split-precision (INT8 MFMA, Ozaki scheme) dgemm.

* Slicing: exponents and int8 slices equal the reference (oracle/ozaki.py) byte for byte.
* Slice products: with alpha = 1, beta = 0 and no intermediate INT32 fold, the result equals the
  reference's recombined sum bit for bit (same exact integer sums, same binary64 order).
* Against the FP64 oracle: max |C - Cref| / D <= 1e-13 with the slice count chosen per exponent
  spread phi (7 for phi = 0, 8 for phi = 8, 10 for phi = 32); integer-valued inputs are exact.
"""
import itertools

import numpy as np
import pytest

import oracle.ozaki as oz
import synth
from gpu_util import TOL, check_parity, logical, rel_err, run_oracle, same_bits, sample_indices, \
    sampled_reference

pytestmark = pytest.mark.gpu

TRANS = [a + b for a, b in itertools.product("NT", "NT")]


def _pad3(rows):
    return max(1, rows) + 3


def _op(x, trans, r, c, ld):
    rr, cc = synth.stored_dims(trans, r, c)
    v = synth.view2d(x, rr, cc, ld)
    return v.T if synth.is_trans(trans) else v


def _run_split(p, alpha, beta, S, C=None):
    import paper_1609_00076_amd as mdg
    import torch
    dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    dC = torch.from_numpy(p["C"] if C is None else C).cuda()
    ws_bytes = mdg.mdg_dgemm_split_workspace_size(p["m"], p["n"], p["k"], S)
    ws = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device="cuda")
    st = mdg.mdg_dgemm_split(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, dA,
                             p["lda"], dB, p["ldb"], beta, dC, p["ldc"], S, ws, ws_bytes)
    assert st == 0, mdg.mdg_status_string(st)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def _storage_from_rows(rows_view, operand, trans, pad=5):
    """Column-major storage (with NaN padding) whose op-space rows are rows_view (rows x k):
    op(A) itself for operand 0, op(B)^T for operand 1."""
    opspace = rows_view if operand == 0 else rows_view.T     # op(A) or op(B)
    stored = opspace.T if synth.is_trans(trans) else opspace
    sr, sc = stored.shape
    ld = sr + pad
    X = np.full(ld * sc, np.nan)
    logical(X, sr, sc, ld)[:, :] = stored
    return X, ld


def _slice_byte_index(rp, kp):
    """[r, p] -> byte offset of entry (r, p) within one slice, as the library header states."""
    r = np.arange(rp, dtype=np.int64)[:, None]
    p = np.arange(kp, dtype=np.int64)[None, :]
    i, h = r % 32, (p // 16) % 2
    slot = 2 * i + (h ^ (((i // 4) ^ (i // 8)) & 1))
    idx = (p // 32) * rp * 32 + (r // 32) * 1024 + 16 * slot + p % 16
    assert np.array_equal(np.sort(idx.ravel()), np.arange(rp * kp)), "layout is a permutation"
    return idx


@pytest.mark.parametrize("S", [1, 4, 7, 10])
@pytest.mark.parametrize("operand,trans", [(0, "N"), (0, "T"), (1, "N"), (1, "T")])
def test_slices_match_reference_bytewise(operand, trans, S):
    import paper_1609_00076_amd as mdg
    import torch
    rows, k = 77, 150  # ragged rows, k not a multiple of 64
    rows_view = synth.draw(synth.rng(synth.seed_for(30, S, operand)), rows * k, "scaled",
                           8).reshape(rows, k)
    rows_view[5, :] = 0.0   # a zero row
    rows_view[:, 3] = 0.0   # zero entries
    X, ld = _storage_from_rows(rows_view, operand, trans)
    kp = (k + 63) // 64 * 64
    rp = (rows + 127) // 128 * 128
    want_q, want_e = oz.split_rows(rows_view, S)
    dX = torch.from_numpy(X).cuda()
    sl = torch.full((S * rp * kp,), 99, dtype=torch.int8, device="cuda")
    ex = torch.full((rows,), -999, dtype=torch.int32, device="cuda")
    assert mdg.mdg_split_slices(operand, trans, rows, k, dX, ld, S, sl, ex) == 0
    torch.cuda.synchronize()
    idx = _slice_byte_index(rp, kp)
    got = sl.cpu().numpy().reshape(S, rp * kp)[:, idx]
    assert np.array_equal(ex.cpu().numpy(), want_e.astype(np.int32))
    for s in range(S):
        assert np.array_equal(got[s, :rows, :k], want_q[s]), f"slice {s + 1}"
        assert not np.any(got[s, :rows, k:]), "k padding must be zero"
        assert not np.any(got[s, rows:, :]), "row padding must be zero"


SHAPES = [(1, 1, 1), (17, 33, 5), (64, 64, 64), (65, 63, 130), (130, 70, 200), (200, 129, 64)]


@pytest.mark.parametrize("S", [1, 3, 7, 8, 9, 10])  # both GEMM kernels (up to 8 slices; beyond)
@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_slice_products_match_reference_bitwise(shape, trans, S):
    m, n, k = shape
    p = synth.problem(31, S, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="scaled", phi=8)
    got = logical(_run_split(p, 1.0, 0.0, S), m, n, p["ldc"])
    want = oz.slice_product_sum(_op(p["A"], trans[0], m, k, p["lda"]),
                                _op(p["B"], trans[1], k, n, p["ldb"]), S)
    assert same_bits(got, want)


@pytest.mark.parametrize("S,phi", [(7, 0), (9, 8)])
@pytest.mark.parametrize("trans", ["NN", "TT"])
def test_non_finite_inputs_poison_only_their_row_and_column(S, phi, trans):
    """A NaN in op(A) and an Inf in op(B): the oracle's C is non-finite exactly on that row of C
    and that column of C; the split path gives NaN there and the oracle's values (to 1e-13 of D)
    everywhere else. The exponent-only entry point flags both lines."""
    import paper_1609_00076_amd as mdg
    import torch
    ta, tb = trans
    m, n, k = 150, 90, 200
    p = synth.problem(36, S, ta, tb, m, n, k, ld_rule=_pad3, dist="scaled" if phi else "uniform",
                      phi=phi)
    ia, pa, jb, pb = 37, 11, 61, 150
    opa = _op(p["A"], ta, m, k, p["lda"])
    opb = _op(p["B"], tb, k, n, p["ldb"])
    opa[ia, pa] = np.nan    # a view into p["A"]'s storage
    opb[pb, jb] = np.inf
    got = logical(_run_split(p, 1.0, 0.5, S), m, n, p["ldc"])
    ref_full, D = run_oracle(p, 1.0, 0.5)
    ref = logical(ref_full, m, n, p["ldc"])
    bad = ~np.isfinite(ref)
    expect_bad = np.zeros((m, n), bool)
    expect_bad[ia, :] = True
    expect_bad[:, jb] = True
    assert np.array_equal(bad, expect_bad), "the oracle's non-finite pattern (a pin of the test)"
    assert np.all(np.isnan(got[bad]))
    Dm = D.reshape(n, m).T
    assert rel_err(got[~bad], ref[~bad], Dm[~bad]) <= TOL
    # the slicing entry point reports both lines as non-finite
    for operand, trans_x, X, ld, rows, line in ((0, ta, p["A"], p["lda"], m, ia),
                                                 (1, tb, p["B"], p["ldb"], n, jb)):
        dX = torch.from_numpy(X).cuda()
        kp = (k + 63) // 64 * 64
        rp = (rows + 127) // 128 * 128
        sl = torch.empty(S * rp * kp, dtype=torch.int8, device="cuda")
        ex = torch.empty(rows, dtype=torch.int32, device="cuda")
        assert mdg.mdg_split_slices(operand, trans_x, rows, k, dX, ld, S, sl, ex) == 0
        torch.cuda.synchronize()
        e = ex.cpu().numpy()
        assert e[line] == 0x7FFFFFFF and np.all(np.delete(e, line) < 64)


@pytest.mark.parametrize("phi,S", [(0, 7), (8, 8), (32, 10)])
@pytest.mark.parametrize("trans", TRANS)
def test_against_fp64_oracle(trans, phi, S):
    m, n, k = 190, 170, 300
    dist = "scaled" if phi else "uniform"
    p = synth.problem(32, phi, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist=dist, phi=phi)
    got = _run_split(p, -0.75, 1.25, S)
    ref, D = run_oracle(p, -0.75, 1.25)
    e = rel_err(logical(got, m, n, p["ldc"]).T, logical(ref, m, n, p["ldc"]).T, D)
    assert e <= TOL, f"split error {e:.2e} (phi={phi}, S={S})"
    pad = got.view(np.uint64).reshape(n, p["ldc"])[:, m:]
    assert np.all(pad == synth.PAD_C_BITS)


@pytest.mark.parametrize("S", [1, 7])
def test_integer_inputs_are_exact(S):
    p = synth.problem(33, S, "T", "N", 150, 140, 222, ld_rule=_pad3, dist="int")
    got = _run_split(p, 1.5, 0.5, S)
    ref, _ = run_oracle(p, 1.5, 0.5)
    assert same_bits(logical(got, 150, 140, p["ldc"]), logical(ref, 150, 140, p["ldc"]))


# INT32 sums are folded into FP64 before they could overflow: for 10 slices every 208 k-steps of
# 64 (k = 13312), for 8 slices every 520 k-steps of 32 (k = 16640); each k below crosses a fold.
@pytest.mark.parametrize("S,k,phi", [(10, 14000, 32), (8, 17000, 8)])
def test_int32_fold_path_long_k(S, k, phi):
    p = synth.problem(34, 0, "N", "T", 80, 72, k, ld_rule=_pad3, dist="scaled", phi=phi)
    got = _run_split(p, 1.0, 1.0, S)
    ref, D = run_oracle(p, 1.0, 1.0)
    assert rel_err(logical(got, 80, 72, p["ldc"]).T, logical(ref, 80, 72, p["ldc"]).T, D) <= TOL


def test_zero_rules_and_errors():
    import paper_1609_00076_amd as mdg
    import torch
    p = synth.problem(35, 0, "N", "N", 40, 30, 20, ld_rule=_pad3)
    C = p["C"].copy()
    logical(C, 40, 30, p["ldc"])[:, :] = np.nan
    got = _run_split(p, 1.0, 0.0, 7, C=C)  # beta = 0 ignores NaN in C
    assert np.all(np.isfinite(logical(got, 40, 30, p["ldc"])))
    dC = torch.from_numpy(p["C"].copy()).cuda()
    # alpha = 0: C := beta*C without slices or workspace
    assert mdg.mdg_dgemm_split("N", "N", 40, 30, 20, 0.0, None, p["lda"], None, p["ldb"], 2.0, dC,
                               p["ldc"], 7, None, 0) == 0
    assert np.array_equal(logical(dC.cpu().numpy(), 40, 30, p["ldc"]),
                          2.0 * logical(p["C"], 40, 30, p["ldc"]))
    dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    need = mdg.mdg_dgemm_split_workspace_size(40, 30, 20, 7)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    args = ("N", "N", 40, 30, 20, 1.0, dA, p["lda"], dB, p["ldb"], 0.0, dC, p["ldc"])
    assert mdg.mdg_dgemm_split(*args, 0, ws, need) == 14
    assert mdg.mdg_dgemm_split(*args, mdg.mdg_split_max_slices() + 1, ws, need) == 14
    assert mdg.mdg_dgemm_split(*args, 7, ws, need - 1) == 15
    assert mdg.mdg_dgemm_split(*args, 7, ws.data_ptr() + 8, need) == 15  # misaligned
    assert mdg.mdg_dgemm_split(*args, 7, None, need) == 15
    assert mdg.mdg_dgemm_split_workspace_size(40, 30, 20, 0) == -1


@pytest.mark.parametrize("phi,S", [(0, 7), (8, 8), (32, 10)])
def test_8192_sampled(phi, S):
    """The split workload at full size: NN, m = n = k = 8192, entries u*2^e, e ~ U{-phi..phi}."""
    import paper_1609_00076_amd as mdg
    import torch
    m = n = k = 8192
    dist = "scaled" if phi else "uniform"
    p = synth.problem(3, phi, "N", "N", m, n, k, ld_rule=synth.ld_round8, dist=dist, phi=phi)
    print(f"[split] 8192^3 phi={phi} S={S}", flush=True)
    dA, dB, dC = (torch.from_numpy(p[x]).cuda() for x in "ABC")
    ws_bytes = mdg.mdg_dgemm_split_workspace_size(m, n, k, S)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    assert mdg.mdg_dgemm_split("N", "N", m, n, k, 1.0, dA, p["lda"], dB, p["ldb"], 1.0, dC,
                               p["ldc"], S, ws, ws_bytes) == 0
    torch.cuda.synchronize()
    R = sample_indices(m, 10, synth.seed_for(3, phi, 5))
    Sx = sample_indices(n, 10, synth.seed_for(3, phi, 6))
    c2 = dC.view(n, p["ldc"])
    got_rows = c2[:, torch.from_numpy(R).cuda()].T.cpu().numpy()
    got_cols = c2[torch.from_numpy(Sx).cuda(), :m].T.cpu().numpy()
    del dA, dB, dC, ws, c2
    ref_r, d_r, ref_c, d_c = sampled_reference(p, 1.0, 1.0, R, Sx)
    er, ec = rel_err(got_rows, ref_r, d_r), rel_err(got_cols, ref_c, d_c)
    print(f"[split] phi={phi} S={S} row err {er:.2e} col err {ec:.2e}", flush=True)
    assert er <= TOL and ec <= TOL


@pytest.mark.parametrize("S,trans", [(9, "TN"), (10, "NT")])
def test_wide_slice_kernel_at_size(S, trans):
    """The 64x64-tile kernel that runs 9 and 10 slices (the served stream's phi = 8 requests use
    9), at a ragged size near the top of the served range, on sampled full rows and columns."""
    import paper_1609_00076_amd as mdg
    import torch
    m, n, k = 2500, 1900, 3100
    p = synth.problem(37, S, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="scaled", phi=8)
    print(f"[split] {trans} {m}x{n}x{k} S={S}", flush=True)
    dA, dB, dC = (torch.from_numpy(p[x]).cuda() for x in "ABC")
    ws_bytes = mdg.mdg_dgemm_split_workspace_size(m, n, k, S)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    assert mdg.mdg_dgemm_split(trans[0], trans[1], m, n, k, -0.75, dA, p["lda"], dB, p["ldb"], 0.5,
                               dC, p["ldc"], S, ws, ws_bytes) == 0
    torch.cuda.synchronize()
    got = logical(dC.cpu().numpy(), m, n, p["ldc"])
    R = sample_indices(m, 12, synth.seed_for(37, S, 5))
    Sx = sample_indices(n, 12, synth.seed_for(37, S, 6))
    ref_r, d_r, ref_c, d_c = sampled_reference(p, -0.75, 0.5, R, Sx)
    er, ec = rel_err(got[R, :], ref_r, d_r), rel_err(got[:, Sx], ref_c, d_c)
    print(f"[split] S={S} row err {er:.2e} col err {ec:.2e}", flush=True)
    assert er <= TOL and ec <= TOL

"""GPU parity of the split-precision dgemm by the Chinese remainder theorem (Ozaki scheme II).

* Residues: the int8 residues of the scaled integers equal the reference (oracle/ozaki.py) byte
  for byte, for both operands, both storage orders, several widths and modulus counts.
* The whole call with alpha = 1, beta = 0 equals the reference's RN(X) 2^(e_i + f_j - 2w) bit for
  bit (X the exact integer product, recovered by CRT; one rounding).
* Against the FP64 oracle: max |C - Cref| / D <= 1e-13 with 14 / 15 / 18 moduli for exponent spreads
  0 / 8 / 32 at k = 700 (16 for spread 32 at k = 8192), on ragged shapes in every transpose case
  with general alpha and beta; integer-valued inputs are exact; 8192^3 on sampled rows and columns.
"""
import itertools

import numpy as np
import pytest

import oracle.ozaki as oz
import synth
from gpu_util import TOL, logical, rel_err, run_oracle, same_bits, sample_indices, \
    sampled_reference

pytestmark = pytest.mark.gpu

TRANS = [a + b for a, b in itertools.product("NT", "NT")]


def _pad3(rows):
    return max(1, rows) + 3


def _op(x, trans, r, c, ld):
    rr, cc = synth.stored_dims(trans, r, c)
    v = synth.view2d(x, rr, cc, ld)
    return v.T if synth.is_trans(trans) else v


def _run_crt(p, alpha, beta, nmod, C=None):
    import paper_1609_00076_amd as mdg
    import torch
    dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    dC = torch.from_numpy(p["C"] if C is None else C).cuda()
    ws_bytes = mdg.mdg_dgemm_crt_workspace_size(p["m"], p["n"], p["k"], nmod)
    ws = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device="cuda")
    st = mdg.mdg_dgemm_crt(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, dA, p["lda"],
                           dB, p["ldb"], beta, dC, p["ldc"], nmod, ws, ws_bytes)
    assert st == 0, mdg.mdg_status_string(st)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def _storage_from_rows(rows_view, operand, trans, pad=5):
    opspace = rows_view if operand == 0 else rows_view.T
    stored = opspace.T if synth.is_trans(trans) else opspace
    sr, sc = stored.shape
    ld = sr + pad
    X = np.full(ld * sc, np.nan)
    logical(X, sr, sc, ld)[:, :] = stored
    return X, ld


def _slice_byte_index(rp, kp):
    r = np.arange(rp, dtype=np.int64)[:, None]
    p = np.arange(kp, dtype=np.int64)[None, :]
    i, h = r % 32, (p // 16) % 2
    slot = 2 * i + (h ^ (((i // 4) ^ (i // 8)) & 1))
    return (p // 32) * rp * 32 + (r // 32) * 1024 + 16 * slot + p % 16


@pytest.mark.parametrize("nmod,bits", [(1, 5), (8, 30), (16, 55), (24, 72)])
@pytest.mark.parametrize("operand,trans", [(0, "N"), (0, "T"), (1, "N"), (1, "T")])
def test_residues_match_reference_bytewise(operand, trans, nmod, bits):
    import paper_1609_00076_amd as mdg
    import torch
    rows, k = 77, 150
    rows_view = synth.draw(synth.rng(synth.seed_for(60, nmod, operand)), rows * k, "scaled",
                           8).reshape(rows, k)
    rows_view[5, :] = 0.0
    rows_view[:, 3] = 0.0
    rows_view[9, 7] = -rows_view[9, 7]
    X, ld = _storage_from_rows(rows_view, operand, trans)
    kp = (k + 63) // 64 * 64
    rp = (rows + 127) // 128 * 128
    dX = torch.from_numpy(X).cuda()
    res = torch.full((nmod * rp * kp,), 77, dtype=torch.int8, device="cuda")
    ex = torch.zeros(rows, dtype=torch.int32, device="cuda")
    assert mdg.mdg_crt_residues(operand, trans, rows, k, dX, ld, nmod, bits, res, ex) == 0
    torch.cuda.synchronize()
    got = res.cpu().numpy().reshape(nmod, rp * kp)
    assert np.array_equal(ex.cpu().numpy(), oz.row_exponents(rows_view))
    Xi, _ = oz.to_integers(rows_view, bits)
    want = oz.crt_residue_matrices(Xi, nmod)
    idx = _slice_byte_index(rp, kp)
    for l in range(nmod):
        full = np.zeros((rp, kp), dtype=np.int64)
        full[:rows, :k] = want[l]
        assert np.array_equal(got[l][idx].astype(np.int64), full), f"modulus {l}"


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape,nmod", [((70, 50, 90), 14), ((257, 129, 65), 16), ((33, 300, 31), 20)])
def test_whole_call_equals_reference_bitwise(shape, nmod, trans):
    m, n, k = shape
    p = synth.problem(61, nmod, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="scaled", phi=8)
    got = logical(_run_crt(p, 1.0, 0.0, nmod), m, n, p["ldc"])
    want = oz.crt_emulated(_op(p["A"], trans[0], m, k, p["lda"]),
                           _op(p["B"], trans[1], k, n, p["ldb"]), nmod)
    assert same_bits(got, want)


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("phi,nmod", [(0, 14), (8, 15), (32, 18)])
def test_against_fp64_oracle(trans, phi, nmod):
    """(At k = 700 an exponent spread of 32 needs 18 moduli; 16 suffice from k ~ 2048 on.)"""
    m, n, k = 300, 190, 700
    dist = "scaled" if phi else "uniform"
    p = synth.problem(62, phi, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist=dist, phi=phi)
    got = _run_crt(p, -0.75, 1.5, nmod)
    ref, D = run_oracle(p, -0.75, 1.5)
    e = rel_err(logical(got, m, n, p["ldc"]).T, logical(ref, m, n, p["ldc"]).T, D)
    assert e <= TOL, f"{trans} phi={phi} nmod={nmod}: {e:.2e}"
    pad = got.view(np.uint64).reshape(n, p["ldc"])[:, m:]
    assert np.all(pad == synth.PAD_C_BITS)


@pytest.mark.parametrize("nmod", [8, 16])
def test_integer_inputs_are_exact(nmod):
    p = synth.problem(63, nmod, "T", "N", 190, 150, 260, ld_rule=_pad3, dist="int")
    got = _run_crt(p, 1.5, 0.5, nmod)
    ref, _ = run_oracle(p, 1.5, 0.5)
    assert same_bits(logical(got, 190, 150, p["ldc"]), logical(ref, 190, 150, p["ldc"]))


def test_long_k_folds_the_accumulators():
    """k beyond 2^17: the INT32 accumulators are reduced modulo m_l on the way."""
    m, n, k = 40, 36, 140000
    p = synth.problem(64, 0, "N", "T", m, n, k, ld_rule=_pad3, dist="scaled", phi=8)
    got = _run_crt(p, 1.0, 1.0, 18)
    ref, D = run_oracle(p, 1.0, 1.0)
    assert rel_err(logical(got, m, n, p["ldc"]).T, logical(ref, m, n, p["ldc"]).T, D) <= TOL


def test_zero_rules_errors_and_non_finite():
    import paper_1609_00076_amd as mdg
    import torch
    p = synth.problem(65, 0, "N", "N", 40, 30, 20, ld_rule=_pad3)
    C = p["C"].copy()
    logical(C, 40, 30, p["ldc"])[:, :] = np.nan
    got = _run_crt(p, 1.0, 0.0, 14, C=C)  # beta = 0 ignores NaN in C
    assert np.all(np.isfinite(logical(got, 40, 30, p["ldc"])))
    dC = torch.from_numpy(p["C"].copy()).cuda()
    assert mdg.mdg_dgemm_crt("N", "N", 40, 30, 20, 0.0, None, p["lda"], None, p["ldb"], 2.0, dC,
                             p["ldc"], 14, None, 0) == 0
    torch.cuda.synchronize()
    assert np.array_equal(logical(dC.cpu().numpy(), 40, 30, p["ldc"]),
                          2.0 * logical(p["C"], 40, 30, p["ldc"]))
    dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    need = mdg.mdg_dgemm_crt_workspace_size(40, 30, 20, 14)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    args = ("N", "N", 40, 30, 20, 1.0, dA, p["lda"], dB, p["ldb"], 0.0, dC, p["ldc"])
    assert mdg.mdg_dgemm_crt(*args, 0, ws, need) == 14
    assert mdg.mdg_dgemm_crt(*args, mdg.mdg_crt_max_moduli() + 1, ws, need) == 14
    assert mdg.mdg_dgemm_crt(*args, 14, ws, need - 1) == 15
    assert mdg.mdg_dgemm_crt(*args, 14, ws.data_ptr() + 8, need) == 15
    # a NaN in op(A) row 7 and an Inf in op(B) column 4: NaN exactly there, the oracle elsewhere
    q = synth.problem(66, 0, "N", "N", 120, 70, 90, ld_rule=_pad3)
    _op(q["A"], "N", 120, 90, q["lda"])[7, 11] = np.nan
    _op(q["B"], "N", 90, 70, q["ldb"])[30, 4] = np.inf
    got = logical(_run_crt(q, 1.0, 0.5, 14), 120, 70, q["ldc"])
    ref_full, D = run_oracle(q, 1.0, 0.5)
    ref = logical(ref_full, 120, 70, q["ldc"])
    bad = ~np.isfinite(ref)
    assert bad[7, :].all() and bad[:, 4].all() and bad.sum() == 70 + 120 - 1
    assert np.all(np.isnan(got[bad]))
    assert rel_err(got[~bad], ref[~bad], D.reshape(70, 120).T[~bad]) <= TOL


@pytest.mark.parametrize("phi,nmod", [(0, 14), (8, 15), (32, 16)])
def test_8192_sampled(phi, nmod):
    import paper_1609_00076_amd as mdg
    import torch
    m = n = k = 8192
    dist = "scaled" if phi else "uniform"
    p = synth.problem(3, phi, "N", "N", m, n, k, ld_rule=synth.ld_round8, dist=dist, phi=phi)
    print(f"[crt] 8192^3 phi={phi} nmod={nmod}", flush=True)
    dA, dB, dC = (torch.from_numpy(p[x]).cuda() for x in "ABC")
    ws_bytes = mdg.mdg_dgemm_crt_workspace_size(m, n, k, nmod)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    assert mdg.mdg_dgemm_crt("N", "N", m, n, k, 1.0, dA, p["lda"], dB, p["ldb"], 1.0, dC,
                             p["ldc"], nmod, ws, ws_bytes) == 0
    torch.cuda.synchronize()
    R = sample_indices(m, 10, synth.seed_for(3, phi, 5))
    Sx = sample_indices(n, 10, synth.seed_for(3, phi, 6))
    c2 = dC.view(n, p["ldc"])
    got_rows = c2[:, torch.from_numpy(R).cuda()].T.cpu().numpy()
    got_cols = c2[torch.from_numpy(Sx).cuda(), :m].T.cpu().numpy()
    del dA, dB, dC, ws, c2
    ref_r, d_r, ref_c, d_c = sampled_reference(p, 1.0, 1.0, R, Sx)
    er, ec = rel_err(got_rows, ref_r, d_r), rel_err(got_cols, ref_c, d_c)
    print(f"[crt] phi={phi} nmod={nmod} row err {er:.2e} col err {ec:.2e}", flush=True)
    assert er <= TOL and ec <= TOL

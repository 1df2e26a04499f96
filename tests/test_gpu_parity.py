"""GPU parity of mdg_dgemm against the CPU oracle at sizes the oracle finishes quickly.

Integer-valued inputs (entries in {-8..8}, alpha and beta multiples of 1/2): every
summation order is exact, so the HIP result must equal the oracle bit for bit.
Uniform[-1,1] inputs: max |C - Cref| / D <= 1e-13 with
D = |alpha| (|op(A)||op(B)|)_ij + |beta||C0_ij|.
Shapes span several macro-tiles of every variant and end in ragged tails in m,
n and k; leading dimensions are rows + 3 (odd, so columns are only 8-byte
aligned) and the padding holds NaN (A, B) or a signalling-NaN pattern (C).
"""
import itertools

import numpy as np
import pytest

import synth
from gpu_util import check_parity, logical, rel_err, run_mdg, run_oracle, same_bits

pytestmark = pytest.mark.gpu

TRANS = [a + b for a, b in itertools.product("NT", "NT")]


def _variants():
    import paper_1609_00076_amd as mdg
    return [-1] + list(range(mdg.mdg_num_variants()))


VARIANTS = _variants()

SHAPES = [(1, 1, 1), (1, 17, 3), (17, 1, 5), (5, 7, 1), (16, 16, 4), (64, 64, 16), (65, 63, 17),
          (128, 128, 16), (129, 130, 31), (200, 300, 77), (255, 257, 129), (300, 200, 513)]


def _pad3(rows):
    return max(1, rows) + 3


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("trans", TRANS)
def test_workload_256_float(trans, variant):
    """m = n = k = 256, ld = 260, alpha = 1.5, beta = 0.5, Uniform[-1,1] entries."""
    p = synth.problem(1, 0, trans[0], trans[1], 256, 256, 256, ld_rule=lambda r: 260)
    check_parity(p, 1.5, 0.5, variant)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("trans", TRANS)
def test_workload_256_integer_bit_exact(trans, variant):
    p = synth.problem(1, 1, trans[0], trans[1], 256, 256, 256, ld_rule=lambda r: 260, dist="int")
    check_parity(p, 1.5, 0.5, variant, exact=True)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ragged_integer_bit_exact(shape, trans, variant):
    m, n, k = shape
    p = synth.problem(10, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="int")
    check_parity(p, 1.5, -0.5, variant, exact=True)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ragged_float(shape, trans, variant):
    m, n, k = shape
    p = synth.problem(11, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
    check_parity(p, -0.75, 1.25, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_beta_zero_never_reads_c(variant):
    p = synth.problem(12, 0, "N", "T", 150, 97, 40, ld_rule=_pad3)
    C = p["C"].copy()
    logical(C, 150, 97, p["ldc"])[:, :] = np.nan
    got = check_parity(p, 2.0, 0.0, variant, C=C)
    assert np.all(np.isfinite(logical(got, 150, 97, p["ldc"])))


@pytest.mark.parametrize("beta", [0.0, 1.0, -2.5])
def test_alpha_zero_and_k_zero(beta):
    import paper_1609_00076_amd as mdg
    import torch
    m, n = 77, 45
    p = synth.problem(13, 0, "N", "N", m, n, 9, ld_rule=_pad3)
    for alpha, k in ((0.0, 9), (1.0, 0)):
        C0 = p["C"].copy()
        dC = torch.from_numpy(C0).cuda()
        # A and B are never read on this path: pass NULL
        st = mdg.mdg_dgemm("N", "N", m, n, k, alpha, None, p["lda"], None, p["ldb"], beta, dC,
                           p["ldc"])
        assert st == 0
        got = dC.cpu().numpy()
        want = beta * logical(p["C"], m, n, p["ldc"]) if beta != 0 else np.zeros((m, n))
        assert np.array_equal(logical(got, m, n, p["ldc"]), want)
        assert np.array_equal(got.view(np.uint64).reshape(n, -1)[:, m:],
                              p["C"].view(np.uint64).reshape(n, -1)[:, m:])


def test_nan_in_a_poisons_one_row():
    for trans in TRANS:
        m, n, k = 140, 70, 50
        p = synth.problem(14, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
        r, c = synth.stored_dims(trans[0], m, k)
        st = logical(p["A"], r, c, p["lda"])
        i0, q0 = 131, 17
        if trans[0] == "T":
            st[q0, i0] = np.nan
        else:
            st[i0, q0] = np.nan
        got = logical(run_mdg(p, 1.0, 1.0), m, n, p["ldc"])
        want = np.zeros((m, n), dtype=bool)
        want[i0, :] = True
        assert np.array_equal(np.isnan(got), want), trans


def test_all_variants_agree_bitwise_on_integer_data():
    p = synth.problem(15, 0, "T", "N", 333, 277, 191, ld_rule=_pad3, dist="int")
    outs = [run_mdg(p, 0.5, 1.5, v) for v in VARIANTS]
    for o in outs[1:]:
        assert same_bits(o, outs[0])


def test_binding_rejects_short_storage():
    import paper_1609_00076_amd as mdg
    import torch
    a = torch.zeros(10, dtype=torch.float64, device="cuda")
    c = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        mdg.mdg_dgemm("N", "N", 4, 4, 4, 1.0, a, 4, a, 4, 0.0, c, 4)
    with pytest.raises(TypeError):
        mdg.mdg_dgemm("N", "N", 2, 2, 2, 1.0, a.float(), 2, a, 2, 0.0, c, 2)


def test_runs_on_a_side_stream():
    import paper_1609_00076_amd as mdg
    import torch
    p = synth.problem(16, 0, "N", "N", 257, 129, 65, ld_rule=_pad3, dist="int")
    dA, dB, dC = (torch.from_numpy(p[x]).cuda() for x in "ABC")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert mdg.mdg_dgemm("N", "N", 257, 129, 65, 1.0, dA, p["lda"], dB, p["ldb"], 1.0, dC,
                             p["ldc"], stream=s) == 0
    s.synchronize()
    ref, _ = run_oracle(p, 1.0, 1.0)
    assert same_bits(logical(dC.cpu().numpy(), 257, 129, p["ldc"]), logical(ref, 257, 129, p["ldc"]))


def test_concurrent_host_threads_on_separate_streams():
    """The library is reentrant: four host threads, each with its own stream and problems, call
    mdg_dgemm at the same time; every result matches the oracle bitwise (integer data)."""
    import threading

    import paper_1609_00076_amd as mdg
    import torch
    shapes = [(300, 200, 150), (129, 257, 64), (64, 64, 300), (500, 70, 33)]
    probs = [synth.problem(17, i, "NT"[i % 2], "TN"[i // 2 % 2], m, n, k, ld_rule=_pad3, dist="int")
             for i, (m, n, k) in enumerate(shapes)]
    dev = [tuple(torch.from_numpy(p[x]).cuda() for x in "ABC") for p in probs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in probs]
    status = [None] * len(probs)
    barrier = threading.Barrier(len(probs))

    def work(i):
        p, (dA, dB, dC) = probs[i], dev[i]
        barrier.wait()
        sts = []
        for _ in range(3):  # C := 1.0*op(A)op(B) + 0.5*C, three times on the same stream
            sts.append(mdg.mdg_dgemm(p["transa"], p["transb"], p["m"], p["n"], p["k"], 1.0, dA,
                                     p["lda"], dB, p["ldb"], 0.5, dC, p["ldc"], stream=streams[i]))
        status[i] = sts

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(probs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for s in streams:
        s.synchronize()
    for i, p in enumerate(probs):
        assert status[i] == [0, 0, 0], status[i]
        ref = p["C"].copy()
        for _ in range(3):
            r, _ = run_oracle(p, 1.0, 0.5, C=ref)
            ref = r
        m, n = p["m"], p["n"]
        assert same_bits(logical(dev[i][2].cpu().numpy(), m, n, p["ldc"]), logical(ref, m, n, p["ldc"]))


@pytest.mark.parametrize("variant", VARIANTS[1:])
def test_transposed_problem_gives_transposed_result_bitwise(variant):
    """C^T = op(B)^T op(A)^T: dgemm(T, T, n, m, k, B, A) on the same storage returns C^T bit for
    bit on Uniform[-1,1] data, for every kernel variant (each variant's k-order does not depend on
    the transpose flags, and the products are the same numbers)."""
    import paper_1609_00076_amd as mdg
    import torch
    m, n, k = 200, 300, 517
    p = synth.problem(18, 0, "N", "N", m, n, k, ld_rule=_pad3)
    dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    C0 = logical(p["C"], m, n, p["ldc"]).copy()          # m x n
    c1 = torch.from_numpy(p["C"].copy()).cuda()
    ldt = n + 3
    ct = np.full(ldt * m, np.nan)
    ct.reshape(m, ldt)[:, :n] = C0                       # C0^T stored column-major, n x m
    c2 = torch.from_numpy(ct).cuda()
    assert mdg.mdg_dgemm_ex(variant, "N", "N", m, n, k, 0.75, dA, p["lda"], dB, p["ldb"], -1.25, c1,
                            p["ldc"]) == 0
    assert mdg.mdg_dgemm_ex(variant, "T", "T", n, m, k, 0.75, dB, p["ldb"], dA, p["lda"], -1.25, c2,
                            ldt) == 0
    torch.cuda.synchronize()
    r1 = logical(c1.cpu().numpy(), m, n, p["ldc"])
    r2 = c2.cpu().numpy().reshape(m, ldt)[:, :n]
    assert same_bits(r1, r2), f"variant {variant}"


@pytest.mark.parametrize("family", [("ring_", "wave_"), ("mfma_",)])
@pytest.mark.parametrize("trans", TRANS)
def test_variant_family_agrees_bitwise_on_float_data(trans, family):
    """Within a kernel family every variant sums each entry's products in the same k-order (ring
    and wave kernels: MFMA k-sets {8s + 2c + e} in order of s and e; register-staged kernels:
    4-deep MFMA steps in order), whatever the tile, wave layout or fragment read; so on
    Uniform[-1,1] data all variants of a family return the same bits."""
    import paper_1609_00076_amd as mdg
    members = [v for v in VARIANTS[1:] if mdg.mdg_variant_name(v).startswith(family)]
    assert len(members) >= 2
    p = synth.problem(19, 0, trans[0], trans[1], 333, 277, 301, ld_rule=_pad3)
    outs = [run_mdg(p, 0.5, 1.5, v) for v in members]
    for v, o in zip(members[1:], outs[1:]):
        assert same_bits(o, outs[0]), f"{mdg.mdg_variant_name(v)} vs {mdg.mdg_variant_name(members[0])}"


@pytest.mark.parametrize("trans", TRANS)
def test_ksplit_k_tails_integer_bit_exact(trans):
    """The k-split ring configurations (two or four wave groups taking alternate 16-deep panels,
    summed in a fixed order at the end): every k around the 32- or 64-deep ring slot (later groups
    with a full, partial or empty last panel, k below one panel) is exact on integer data, and a
    second call returns the same bits on float data."""
    import paper_1609_00076_amd as mdg
    ksplit = [x for x in VARIANTS[1:] if mdg.mdg_variant_name(x).startswith("ringk")]
    assert len(ksplit) == 3
    for v in ksplit:
        for k in (1, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 96, 97, 130):
            p = synth.problem(21, k, trans[0], trans[1], 70, 131, k, ld_rule=_pad3, dist="int")
            check_parity(p, 1.5, -0.5, v, exact=True)
        p = synth.problem(22, 0, trans[0], trans[1], 150, 90, 301, ld_rule=_pad3)
        assert same_bits(run_mdg(p, 0.5, 1.5, v), run_mdg(p, 0.5, 1.5, v))


def oracle_dgemm_dense(a, b, c, alpha, beta):
    """c := alpha * a @ b + beta * c through the oracle (a, b, c dense 2-D arrays, updated in place)."""
    import oracle
    m, k = a.shape
    n = b.shape[1]
    A, B = np.ascontiguousarray(a.T).ravel(), np.ascontiguousarray(b.T).ravel()
    C = np.ascontiguousarray(c.T).ravel()
    st = oracle.dgemm("N", "N", m, n, k, alpha, A, m, B, k, beta, C, m)
    c[:, :] = C.reshape(n, m).T
    return st == 0


def test_leading_dimensions_at_the_offset_limit():
    """Leading dimensions just inside what the kernels' 32-bit panel offsets address: a 16-deep
    k-panel of an operand strided along k spans 15 * ld + 256 elements, just under 4 GiB of bytes.
    Every variant computes the GEMM exactly (integer data, NaN in every element outside the
    matrices), for op(A) and for op(B) strided along k; a slightly larger ld is refused on the host."""
    import paper_1609_00076_amd as mdg
    import torch
    m, n, k = 70, 50, 40
    ld = (((1 << 32) - 16) // 8 - 256) // 15            # 15 * ld + 256 elements fit 32-bit byte offsets
    assert (15 * ld + 256) * 8 + 16 <= (1 << 32) < (15 * (ld + 20) + 256) * 8 + 16
    g = synth.rng(synth.seed_for(20, 0, 0))
    a = g.integers(-8, 9, (m, k)).astype(np.float64)     # op(A), m x k
    b = g.integers(-8, 9, (k, n)).astype(np.float64)     # op(B), k x n
    c0 = g.integers(-8, 9, (m, n)).astype(np.float64)
    want = c0.copy()
    assert oracle_dgemm_dense(a, b, want, 1.5, 0.5)
    dA = torch.full((k * ld,), float("nan"), dtype=torch.float64, device="cuda")
    dA.view(k, ld)[:, :m] = torch.from_numpy(a.T.copy()).cuda()          # A stored m x k, lda = ld
    dBt = torch.full((k * ld,), float("nan"), dtype=torch.float64, device="cuda")
    dBt.view(k, ld)[:, :n] = torch.from_numpy(b.copy()).cuda()           # B stored n x k, ldb = ld
    dA_small = torch.from_numpy(a.T.copy().ravel()).cuda()               # A stored m x k, lda = m
    dB_small = torch.from_numpy(b.T.copy().ravel()).cuda()               # B stored k x n, ldb = k
    for v in VARIANTS:
        for tb, B, ldb, A, lda in (("N", dB_small, k, dA, ld), ("T", dBt, ld, dA_small, m)):
            dC = torch.from_numpy(c0.T.copy().ravel()).cuda()
            st = mdg.mdg_dgemm_ex(v, "N", tb, m, n, k, 1.5, A, lda, B, ldb, 0.5, dC, m)
            assert st == 0, (v, tb, mdg.mdg_status_string(st))
            torch.cuda.synchronize()
            got = dC.cpu().numpy().reshape(n, m).T
            assert same_bits(got, want), f"variant {v} transb {tb}"
    big = [v for v in VARIANTS[1:] if mdg.mdg_variant_name(v) == "ring_f64_256x128x16_w128x32_s3_il"][0]
    dC = torch.from_numpy(c0.T.copy().ravel()).cuda()
    assert mdg.mdg_dgemm_ex(big, "N", "N", m, n, k, 1.5, dA, ld + 20, dB_small, k, 0.5, dC, m) == -4


@pytest.mark.parametrize("layouts", ["colcolcol", "rowrowrow", "colrowcol", "rowcolrow"])
@pytest.mark.parametrize("trans", TRANS)
def test_gemm2d_tensor_form(layouts, trans):
    """gemm2d on 2-D device tensors (column-major with padded ld, or row-major) equals the
    oracle's result of the same GEMM bit for bit on integer data."""
    import paper_1609_00076_amd as mdg
    import torch
    la, lb, lc = layouts[:3], layouts[3:6], layouts[6:]
    m, n, k = 150, 97, 70
    g = synth.rng(synth.seed_for(31, 0, 0))
    opa = g.integers(-8, 9, (m, k)).astype(np.float64)
    opb = g.integers(-8, 9, (k, n)).astype(np.float64)
    c0 = g.integers(-8, 9, (m, n)).astype(np.float64)

    def dev(x, layout, pad):
        r, c = x.shape
        if layout == "col":
            base = torch.full((c, r + pad), float("nan"), dtype=torch.float64, device="cuda")
            view = base[:, :r].t()
        else:
            base = torch.full((r, c + pad), float("nan"), dtype=torch.float64, device="cuda")
            view = base[:, :c]
        view.copy_(torch.from_numpy(x))
        return view

    A = dev(opa.T.copy() if trans[0] == "T" else opa, la, 3)
    B = dev(opb.T.copy() if trans[1] == "T" else opb, lb, 5)
    C = dev(c0, lc, 2)
    mdg.gemm2d(A, B, C, 1.5, -0.5, trans[0], trans[1])
    assert oracle_dgemm_dense(opa, opb, c0, 1.5, -0.5)  # c0 := the oracle's result
    assert same_bits(C.cpu().numpy(), c0)

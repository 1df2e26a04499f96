"""GPU parity of the thin kernel and of split plans (tiled block + thin fringes) against the oracle.

A C with at most 16 rows or columns is computed by the thin kernel alone; a C whose m or n exceeds
a multiple of a big tile by at most 16 is computed as the tiled block plus one thin launch for the
fringe rows and columns (paper, section 2.4). Each test first checks, through mdg_dgemm_plan, that
the automatic dgemm takes the path it is meant to exercise, then compares with the oracle:
bit-exact on integer-valued inputs, within 1e-13 of |alpha| |op(A)||op(B)| + |beta||C| on uniform
inputs; padding rows of C (a signalling-NaN pattern) must be left untouched.
"""
import itertools

import numpy as np
import pytest

import synth
from gpu_util import (TOL, check_parity, logical, padding_untouched, rel_err, run_mdg,
                      sample_indices, sampled_reference, same_bits)

pytestmark = pytest.mark.gpu

TRANS = [a + b for a, b in itertools.product("NT", "NT")]

# thin side 1..16 (every kernel bucket: <= 4, <= 8, <= 16), rows form and columns form, k ragged
# against the 256-deep chunks, long side ragged against the 16 outputs of a workgroup
THIN = [(3, 4099, 700), (1, 1500, 300), (16, 2100, 257), (9, 1100, 1000), (5, 3000, 513),
        (2000, 3, 600), (1200, 16, 300), (3001, 7, 256), (4, 4, 4000), (1, 1, 5000),
        (16, 300, 2000)]
# tiled block plus thin fringe rows, columns or both
SPLIT = [(1025, 1024, 1024), (1030, 2000, 700), (2056, 1030, 900), (3075, 2050, 500)]


def _pad3(rows):
    return max(1, rows) + 3


def _plan(trans, m, n, k):
    import paper_1609_00076_amd as mdg
    return mdg.mdg_dgemm_plan(trans[0], trans[1], m, n, k)


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", THIN, ids=lambda s: "x".join(map(str, s)))
def test_thin_only_integer_bit_exact(shape, trans):
    m, n, k = shape
    assert _plan(trans, m, n, k)[0] == -1
    p = synth.problem(30, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="int")
    print(f"[thin] {trans} {m}x{n}x{k} integer", flush=True)
    check_parity(p, 1.5, -0.5, exact=True)


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", THIN, ids=lambda s: "x".join(map(str, s)))
def test_thin_only_float(shape, trans):
    m, n, k = shape
    p = synth.problem(31, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
    print(f"[thin] {trans} {m}x{n}x{k} uniform", flush=True)
    check_parity(p, -0.75, 1.25)


@pytest.mark.parametrize("trans", TRANS)
def test_thin_beta_zero_never_reads_c(trans):
    for m, n, k in ((5, 700, 300), (700, 5, 300)):
        p = synth.problem(32, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
        C = p["C"].copy()
        logical(C, m, n, p["ldc"])[:, :] = np.nan
        got = check_parity(p, 2.0, 0.0, C=C)
        assert np.all(np.isfinite(logical(got, m, n, p["ldc"])))


def test_thin_nan_in_a_poisons_one_row():
    """A NaN in row i0 of op(A) reaches row i0 of C only (zeros past k or past the long side
    are not multiplied into real outputs)."""
    for trans in TRANS:
        m, n, k = 6, 900, 530
        p = synth.problem(33, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
        r, c = synth.stored_dims(trans[0], m, k)
        st = logical(p["A"], r, c, p["lda"])
        i0, q0 = 4, 517
        if trans[0] == "T":
            st[q0, i0] = np.nan
        else:
            st[i0, q0] = np.nan
        got = logical(run_mdg(p, 1.0, 1.0), m, n, p["ldc"])
        want = np.zeros((m, n), dtype=bool)
        want[i0, :] = True
        assert np.array_equal(np.isnan(got), want), trans


@pytest.mark.parametrize("trans", TRANS)
def test_thin_matches_every_tiled_variant_bitwise_on_integer_data(trans):
    """Exact sums: the thin kernel and each tiled variant give the same bits."""
    import paper_1609_00076_amd as mdg
    m, n, k = 7, 1300, 600
    assert _plan(trans, m, n, k)[0] == -1
    p = synth.problem(34, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="int")
    auto = run_mdg(p, 0.5, 1.5)
    for v in range(mdg.mdg_num_variants()):
        assert same_bits(auto, run_mdg(p, 0.5, 1.5, v)), mdg.mdg_variant_name(v)


def _sampled_check(p, alpha, beta, m0, n0, seed):
    """Full rows and columns around the split lines and at the edges, against the oracle."""
    import paper_1609_00076_amd as mdg  # noqa: F401
    m, n = p["m"], p["n"]
    got = logical(run_mdg(p, alpha, beta), m, n, p["ldc"])
    extra_r = [x for x in (m0 - 2, m0 - 1, m0, m0 + 1) if 0 <= x < m]
    extra_c = [x for x in (n0 - 2, n0 - 1, n0, n0 + 1) if 0 <= x < n]
    R = np.array(sorted(set(sample_indices(m, 12, seed).tolist()) | set(extra_r)), dtype=np.int64)
    S = np.array(sorted(set(sample_indices(n, 12, seed + 1).tolist()) | set(extra_c)),
                 dtype=np.int64)
    ref_r, d_r, ref_c, d_c = sampled_reference(p, alpha, beta, R, S)
    return got, R, S, ref_r, d_r, ref_c, d_c


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", SPLIT, ids=lambda s: "x".join(map(str, s)))
def test_split_plan_sampled_float(shape, trans):
    m, n, k = shape
    v, m0, n0 = _plan(trans, m, n, k)
    assert v >= 0 and (m0 < m or n0 < n), (v, m0, n0)
    p = synth.problem(35, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
    print(f"[split] {trans} {m}x{n}x{k} main {m0}x{n0} uniform", flush=True)
    got, R, S, ref_r, d_r, ref_c, d_c = _sampled_check(p, 1.25, -0.5, m0, n0, 36)
    er = rel_err(got[R, :], ref_r, d_r)
    ec = rel_err(got[:, S], ref_c, d_c)
    assert er <= TOL and ec <= TOL, f"row err {er:.2e}, col err {ec:.2e}"


@pytest.mark.parametrize("trans", TRANS)
@pytest.mark.parametrize("shape", SPLIT, ids=lambda s: "x".join(map(str, s)))
def test_split_plan_sampled_integer_bit_exact(shape, trans):
    m, n, k = shape
    v, m0, n0 = _plan(trans, m, n, k)
    assert v >= 0 and (m0 < m or n0 < n), (v, m0, n0)
    p = synth.problem(37, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="int")
    print(f"[split] {trans} {m}x{n}x{k} main {m0}x{n0} integer", flush=True)
    got, R, S, ref_r, _, ref_c, _ = _sampled_check(p, 1.5, 0.5, m0, n0, 38)
    assert same_bits(got[R, :], ref_r) and same_bits(got[:, S], ref_c)


def test_split_plan_whole_matrix_against_the_oracle():
    """One split problem compared in full (every entry, padding untouched)."""
    trans = "TN"
    m, n, k = 1030, 2000, 300
    v, m0, n0 = _plan(trans, m, n, k)
    assert v >= 0 and m0 < m and n0 < n, (v, m0, n0)
    p = synth.problem(39, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3, dist="int")
    check_parity(p, -1.5, 2.0, exact=True)


def test_split_paths_graph_replay_matches_eager():
    """The multi-launch paths (a dgemm split into a tiled block and one thin launch, a thin-only
    dgemm, a dsyrk split into GEMMs and one launch over its diagonal blocks) captured in one graph
    on torch's stream: every replay, with eager work and synchronizations between replays, gives
    the eager results bit for bit."""
    import torch
    import paper_1609_00076_amd as mdg
    from gpu_util import to_dev
    m, n, k = 1030, 2000, 300
    assert _plan("TN", m, n, k)[1:] == (1024, 1984)
    assert _plan("NN", 5, 3000, 513)[0] == -1
    p1 = synth.problem(40, 0, "T", "N", m, n, k, ld_rule=_pad3)
    p2 = synth.problem(40, 1, "N", "N", 5, 3000, 513, ld_rule=_pad3)
    ns, ks = 4096, 40
    hA = synth.matrix(synth.seed_for(40, 2, 0), ns, ks, ns, "uniform")
    hC = synth.matrix(synth.seed_for(40, 2, 1), ns, ns, ns, "uniform")
    d1 = [to_dev(p1[x]) for x in "ABC"]
    d2 = [to_dev(p2[x]) for x in "ABC"]
    dA, dC = to_dev(hA), to_dev(hC)
    inits = [(d1[2], d1[2].clone()), (d2[2], d2[2].clone()), (dC, dC.clone())]

    def calls():
        assert mdg.mdg_dgemm("T", "N", m, n, k, 1.25, d1[0], p1["lda"], d1[1], p1["ldb"], -0.5,
                             d1[2], p1["ldc"]) == 0
        assert mdg.mdg_dgemm("N", "N", 5, 3000, 513, 0.75, d2[0], p2["lda"], d2[1], p2["ldb"], 1.5,
                             d2[2], p2["ldc"]) == 0
        assert mdg.mdg_dsyrk("L", "N", ns, ks, 0.5, dA, ns, 1.5, dC, ns) == 0

    def reset():
        for x, x0 in inits:
            x.copy_(x0)

    calls()  # eager results
    torch.cuda.synchronize()
    want = [x.clone() for x, _ in inits]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # torch's warm-up-before-capture on a side stream
        reset()
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls()
    for rep in range(3):
        reset()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for (got, _), ref in zip(inits, want):
            assert torch.equal(got.view(torch.int64), ref.view(torch.int64)), f"replay {rep}"

"""GPU results at the full sweep sizes, in the launch configuration the benchmark times.

Shapes: square m = n = k in {1024, 2048, 4096, 4099, 8192, 16384} and the skinny
m = n = 8192, k = 64, all four transpose cases, ld = stored rows rounded up to a
multiple of 8, alpha = beta = 1.

The O(mnk) oracle is too slow for whole results here, so two checks stand in:
  * Uniform[-1,1] data: full rows and full columns at edges, tile boundaries and
    random positions are evaluated by the oracle (same products, same order per
    entry) and must agree to 1e-13 relative to D;
  * integer-valued data: Freivalds' identity C x = alpha op(A) (op(B) x) + beta C0 x
    for three seeded integer vectors x. Every quantity is an integer below 2^53, so
    the identity holds exactly, and a wrong entry escapes one vector with
    probability at most 1/17.
"""
import numpy as np
import pytest

import synth
from gpu_util import TOL, logical, rel_err, sample_indices, sampled_reference

pytestmark = pytest.mark.gpu

SHAPES = [(1024,) * 3, (2048,) * 3, (4096,) * 3, (4099,) * 3, (8192, 8192, 64), (8192,) * 3,
          (16384,) * 3]
TRANS = ["NN", "NT", "TN", "TT"]


def _run_device(p, alpha, beta, torch):
    import paper_1609_00076_amd as mdg
    dA = torch.from_numpy(p["A"]).cuda()
    dB = torch.from_numpy(p["B"]).cuda()
    dC = torch.from_numpy(p["C"]).cuda()
    st = mdg.mdg_dgemm(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, dA, p["lda"],
                       dB, p["ldb"], beta, dC, p["ldc"])
    assert st == 0, mdg.mdg_status_string(st)
    torch.cuda.synchronize()
    del dA, dB
    return dC


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_sweep_sampled_rows_and_columns(shape):
    import torch
    m, n, k = shape
    for t, trans in enumerate(TRANS):
        p = synth.problem(2, t, trans[0], trans[1], m, n, k, ld_rule=synth.ld_round8)
        print(f"[sweep] {trans} {m}x{n}x{k} float", flush=True)
        dC = _run_device(p, 1.0, 1.0, torch)
        R = sample_indices(m, 12, synth.seed_for(2, t, 5))
        S = sample_indices(n, 12, synth.seed_for(2, t, 6))
        c2 = dC.view(n, p["ldc"])
        got_rows = c2[:, torch.from_numpy(R).cuda()].T.cpu().numpy()    # |R| x n
        got_cols = c2[torch.from_numpy(S).cuda(), :m].T.cpu().numpy()   # m x |S|
        pad_ok = bool(torch.all(c2[:, m:].contiguous().view(torch.int64)
                                == np.int64(np.uint64(synth.PAD_C_BITS).astype(np.int64))).item()) \
            if p["ldc"] > m else True
        del dC, c2
        ref_r, d_r, ref_c, d_c = sampled_reference(p, 1.0, 1.0, R, S)
        er = rel_err(got_rows, ref_r, d_r)
        ec = rel_err(got_cols, ref_c, d_c)
        assert pad_ok, f"C padding written {trans} {shape}"
        assert er <= TOL and ec <= TOL, f"{trans} {shape}: row err {er:.2e}, col err {ec:.2e}"


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_sweep_integer_freivalds(shape):
    import torch
    m, n, k = shape
    for t, trans in enumerate(TRANS):
        p = synth.problem(2, 10 + t, trans[0], trans[1], m, n, k, ld_rule=synth.ld_round8,
                          dist="int")
        print(f"[sweep] {trans} {m}x{n}x{k} integer", flush=True)
        dC = _run_device(p, 1.0, 1.0, torch)
        C = logical(dC.cpu().numpy(), m, n, p["ldc"])
        del dC
        ra, ca = synth.stored_dims(trans[0], m, k)
        rb, cb = synth.stored_dims(trans[1], k, n)
        A = logical(p["A"], ra, ca, p["lda"])
        B = logical(p["B"], rb, cb, p["ldb"])
        opa = A.T if trans[0] == "T" else A
        opb = B.T if trans[1] == "T" else B
        C0 = logical(p["C"], m, n, p["ldc"])
        g = synth.rng(synth.seed_for(2, 10 + t, 7))
        for _ in range(3):
            x = g.integers(-8, 9, n).astype(np.float64)
            lhs = C @ x
            rhs = opa @ (opb @ x) + C0 @ x
            assert np.array_equal(lhs, rhs), f"Freivalds identity fails: {trans} {shape}"

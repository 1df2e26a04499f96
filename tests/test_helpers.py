"""Test helpers on the CPU: the sampled-entry reference equals the full oracle bitwise."""
import itertools

import numpy as np
import pytest

import synth
from gpu_util import logical, rel_err, run_oracle, same_bits, sample_indices, sampled_reference


@pytest.mark.parametrize("trans", ["NN", "NT", "TN", "TT"])
def test_sampled_reference_matches_full_oracle(trans):
    m, n, k = 300, 270, 45
    p = synth.problem(50, 0, trans[0], trans[1], m, n, k, ld_rule=synth.ld_round8)
    ref, D = run_oracle(p, 0.75, -1.25)
    R = sample_indices(m, 6, 1)
    S = sample_indices(n, 6, 2)
    rr, dr, rc, dc = sampled_reference(p, 0.75, -1.25, R, S)
    full = logical(ref, m, n, p["ldc"])
    Dfull = D.reshape(n, m).T
    assert same_bits(rr, full[R, :]) and same_bits(rc, full[:, S])
    assert same_bits(dr, Dfull[R, :]) and same_bits(dc, Dfull[:, S])
    assert 0 in R and m - 1 in R and 128 in R and n - 1 in S


def test_rel_err_conventions():
    assert rel_err([1.0, 2.0], [1.0, 2.0], [0.0, 1.0]) == 0.0
    assert rel_err([1.0, 2.0], [1.0, 2.5], [1.0, 1.0]) == 0.5
    assert rel_err([1.0], [1.5], [0.0]) == np.inf       # D = 0 requires equality
    assert rel_err([np.nan], [1.0], [1.0]) == np.inf


def test_bench_sampled_oracle_lines_equal_the_full_oracle():
    """bench.py states the split path's error from the oracle's sampled rows and columns; they must
    be the oracle's full-problem values bit for bit (same products, same order)."""
    import numpy as np

    import bench
    import oracle
    import synth
    m, n, k = 300, 200, 150
    p = synth.problem(3, 0, "N", "N", m, n, k, ld_rule=lambda r: r + 5)
    ref = p["C"].copy()
    assert oracle.dgemm("N", "N", m, n, k, 1.0, p["A"], p["lda"], p["B"], p["ldb"], 1.0, ref,
                        p["ldc"]) == 0
    D = np.zeros(m * n)
    assert oracle.absden("N", "N", m, n, k, 1.0, p["A"], p["lda"], p["B"], p["ldb"], 1.0, p["C"],
                         p["ldc"], D, m) == 0
    D = D.reshape(n, m).T
    R, S = bench.sample_lines(m, 4, 1), bench.sample_lines(n, 4, 2)
    assert R[0] == 0 and R[-1] == m - 1 and S[-1] == n - 1
    rr, dr, cc, dc, macs = bench.oracle_lines(p["A"], p["B"], p["C"], m, n, k, p["lda"], p["ldb"],
                                              p["ldc"], 1.0, 1.0, R, S)
    full = synth.view2d(ref, m, n, p["ldc"])
    assert np.array_equal(rr, full[R, :]) and np.array_equal(cc, full[:, S])
    assert np.array_equal(dr, D[R, :]) and np.array_equal(dc, D[:, S])
    assert macs == (len(R) * n + m * len(S)) * k
    assert bench.max_rel_err(cc, full[:, S], dc) == 0.0
    assert bench.max_rel_err(cc + 1e-9, full[:, S], dc) > 0.0

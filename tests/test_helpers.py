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

"""True error of the oracle, the native kernel and the split path, against the doubled-precision
reference (oracle_dgemm_dd, pinned by the dd_* pins in oracle_pins.py).

The parity bar compares the GPU with the plain oracle; this states how far each result is from
the exact product, err = max |C - C_dd| / D with D = |alpha||A||B| + |beta||C0|, on shapes that
span several tiles, a ragged tail and all four transpose cases. Each error is printed; the asserts
are the benchmark spec's bound for the split path and a bound two orders of magnitude above FP64
rounding for the FP64 paths.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, logical, rel_err, run_mdg, run_oracle
from test_gpu_split import _pad3, _run_split

pytestmark = pytest.mark.gpu

TRANS = [a + b for a, b in itertools.product("NT", "NT")]
FP64_BOUND = 1e-14


def _dd(p, alpha, beta):
    C = p["C"].copy()
    assert oracle.dgemm_dd(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, p["A"],
                           p["lda"], p["B"], p["ldb"], beta, C, p["ldc"]) == 0
    return C


@pytest.mark.parametrize("trans", TRANS)
def test_true_error_native_and_oracle(trans):
    m, n, k = 300, 200, 2500
    p = synth.problem(40, 0, trans[0], trans[1], m, n, k, ld_rule=_pad3)
    alpha, beta = 1.25, -0.5
    exact = logical(_dd(p, alpha, beta), m, n, p["ldc"])
    ref, D = run_oracle(p, alpha, beta)
    got = run_mdg(p, alpha, beta)
    e_oracle = rel_err(logical(ref, m, n, p["ldc"]).T, exact.T, D)
    e_native = rel_err(logical(got, m, n, p["ldc"]).T, exact.T, D)
    print(f"[true error] {trans} {m}x{n}x{k}: oracle {e_oracle:.2e}, native {e_native:.2e}")
    assert e_oracle <= FP64_BOUND and e_native <= FP64_BOUND


@pytest.mark.parametrize("phi,S", [(0, 7), (8, 8), (32, 10)])
def test_true_error_split(phi, S):
    m, n, k = 190, 260, 3000
    dist = "scaled" if phi else "uniform"
    p = synth.problem(41, phi, "N", "T", m, n, k, ld_rule=_pad3, dist=dist, phi=phi)
    alpha, beta = 1.0, 1.0
    exact = logical(_dd(p, alpha, beta), m, n, p["ldc"])
    _, D = run_oracle(p, alpha, beta)
    got = _run_split(p, alpha, beta, S)
    e = rel_err(logical(got, m, n, p["ldc"]).T, exact.T, D)
    print(f"[true error] split phi={phi} S={S} {m}x{n}x{k}: {e:.2e}")
    assert e <= TOL

"""The reference of the split-precision scheme (oracle/ozaki.py) against exact facts (CPU only)."""
import numpy as np
import pytest

import oracle
import oracle.ozaki as oz
import synth


def _dense(dist, m, k, seed, phi=0):
    return synth.draw(synth.rng(seed), m * k, dist, phi).reshape(m, k)


def test_exponents_bracket_the_row_maximum():
    X = _dense("scaled", 40, 33, 1, phi=8)
    X[3, :] = 0.0
    e = oz.row_exponents(X)
    mx = np.abs(X).max(axis=1)
    live = mx > 0
    assert np.all(2.0 ** (e[live] - 1) <= mx[live]) and np.all(mx[live] < 2.0 ** e[live])
    assert e[3] == 0


@pytest.mark.parametrize("S", [1, 3, 7, 10])
def test_slices_bounded_and_reconstruct_within_remainder(S):
    X = _dense("scaled", 30, 50, 2, phi=8)
    sl, e = oz.split_rows(X, S)
    assert all(np.abs(q.astype(int)).max() <= 127 for q in sl)
    recon = sum(np.ldexp(q.astype(np.float64), -7 * (s + 1)) for s, q in enumerate(sl))
    scaled = np.ldexp(X, -e[:, None])
    assert np.all(np.abs(scaled - recon) < 2.0 ** (-7 * S))


def test_eight_slices_are_exact_for_entries_near_the_row_maximum():
    # entries with the row maximum's exponent carry 53 bits; 8 slices hold 56
    X = _dense("uniform", 20, 64, 3)
    X = np.where(np.abs(X) < 0.5, X + np.sign(X) * 0.5, X)
    X[:, 0] = 0.999
    sl, e = oz.split_rows(X, 8)
    recon = sum(np.ldexp(q.astype(np.float64), -7 * (s + 1)) for s, q in enumerate(sl))
    assert np.array_equal(np.ldexp(recon, e[:, None]), X)


def test_integer_inputs_fit_one_slice_and_multiply_exactly():
    A = _dense("int", 37, 41, 4)
    B = _dense("int", 41, 29, 5)
    sl, _ = oz.split_rows(A, 4)
    assert all(not np.any(q) for q in sl[1:])
    got = oz.slice_product_sum(A, B, 1)
    assert np.array_equal(got, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


def _err_vs_oracle(A, B, C):
    m, k = A.shape
    n = B.shape[1]
    Af = np.asfortranarray(A).reshape(-1, order="F")
    Bf = np.asfortranarray(B).reshape(-1, order="F")
    ref = np.zeros(m * n)
    assert oracle.dgemm("N", "N", m, n, k, 1.0, Af, m, Bf, k, 0.0, ref, m) == 0
    D = np.zeros(m * n)
    assert oracle.absden("N", "N", m, n, k, 1.0, Af, m, Bf, k, 0.0, ref, m, D, m) == 0
    return float(np.max(np.abs(C - ref.reshape(n, m).T) / D.reshape(n, m).T))


@pytest.mark.parametrize("phi,S", [(0, 7), (8, 8), (32, 10)])
def test_chosen_slice_counts_reach_1e13(phi, S):
    dist = "scaled" if phi else "uniform"
    A = _dense(dist, 96, 160, 6, phi)
    B = _dense(dist, 160, 80, 7, phi)
    assert _err_vs_oracle(A, B, oz.slice_product_sum(A, B, S)) <= 1e-13
    # one slice fewer misses the gate: the count is not padded
    assert _err_vs_oracle(A, B, oz.slice_product_sum(A, B, S - 1)) > 1e-13

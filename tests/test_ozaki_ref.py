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


# ---- scheme II (CRT over int8 moduli) -----------------------------------------------------------

def _exact_int_product(Ai, Bi):
    """A' B'^T of two object arrays of Python ints (rows x k each), in Python integers."""
    m, k = Ai.shape
    n = Bi.shape[0]
    return np.array([[sum(Ai[i, p] * Bi[j, p] for p in range(k)) for j in range(n)]
                     for i in range(m)], dtype=object)


def test_moduli_are_pairwise_coprime_and_fit_int8():
    import math
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(oz.MODULI) for b in oz.MODULI[i + 1:])
    for m in oz.MODULI:
        r = [oz.sym_residue(x, m) for x in range(-3 * m, 3 * m)]
        assert min(r) >= -128 and max(r) <= 127 and len(set(r)) == m
        assert all((x - oz.sym_residue(x, m)) % m == 0 for x in range(-3 * m, 3 * m))


@pytest.mark.parametrize("k,nmod", [(1, 8), (32, 14), (8192, 15), (8192, 20), (3000, 24)])
def test_bits_keep_every_product_inside_half_the_modulus(k, nmod):
    M = oz.crt_modulus(nmod)
    w = oz.crt_bits(k, nmod)
    assert 1 <= w <= oz.MAX_BITS
    assert k * (2 ** w - 1) ** 2 < M // 2          # |A'B'| < M/2 for any k-term dot product
    if w < oz.MAX_BITS:
        assert 4 * k * 2 ** (2 * (w + 1)) > M      # and w is the largest with the margin


@pytest.mark.parametrize("phi,nmod", [(0, 13), (8, 15), (32, 16)])
def test_crt_reconstruction_is_the_exact_integer_product(phi, nmod):
    """Independent of the CRT: the Python-integer product of the scaled integer matrices."""
    dist = "scaled" if phi else "uniform"
    A = _dense(dist, 9, 23, 20 + phi, phi)
    B = _dense(dist, 23, 7, 21 + phi, phi)
    A[2, :] = 0.0                      # a zero row
    A[4, 5:] = -A[4, 5:]               # mixed signs
    X, ea, eb, w = oz.crt_product(A, B, nmod)
    Ai, ea2 = oz.to_integers(A, w)
    Bi, eb2 = oz.to_integers(B.T, w)
    assert np.array_equal(ea, ea2) and np.array_equal(eb, eb2)
    assert all(abs(int(v)) < 2 ** w for v in Ai.ravel()) and all(abs(int(v)) < 2 ** w for v in Bi.ravel())
    want = _exact_int_product(Ai, Bi)
    assert all(int(a) == int(b) for a, b in zip(X.ravel(), want.ravel()))
    assert all(int(v) == 0 for v in X[2, :])


def test_crt_result_is_the_rounded_scaled_integer_product():
    """Step 5 against exact rationals: each entry is the binary64 rounding of the exact scaled
    integer product (one rounding), including a constructed cancellation."""
    from fractions import Fraction
    A = _dense("scaled", 6, 40, 30, 8)
    B = _dense("scaled", 40, 5, 31, 8)
    B[:, 1] = 0.0
    B[0, 1], B[1, 1] = 1.0, 1.0
    A[3, 0], A[3, 1] = 0.75, -0.75 + 2.0 ** -40   # row 3, column 1: a near-total cancellation
    nmod = 16
    C = oz.crt_emulated(A, B, nmod)
    w = oz.crt_bits(40, nmod)
    Ai, ea = oz.to_integers(A, w)
    Bi, eb = oz.to_integers(B.T, w)
    exact = _exact_int_product(Ai, Bi)
    for i in range(6):
        for j in range(5):
            v = Fraction(int(exact[i, j])) * Fraction(2) ** int(ea[i] + eb[j] - 2 * w)
            assert C[i, j] == float(v), (i, j)
    assert C[3, 1] == float(Fraction(0.75) + Fraction(-0.75 + 2.0 ** -40))  # exact here


def test_crt_integer_inputs_are_exact():
    A = _dense("int", 21, 33, 40)
    B = _dense("int", 33, 17, 41)
    got = oz.crt_emulated(A, B, 8)
    assert np.array_equal(got, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


@pytest.mark.parametrize("phi,nmod,k", [(0, 14, 2048), (8, 15, 2048), (32, 16, 2048), (0, 14, 32),
                                        (8, 16, 32)])
def test_chosen_moduli_counts_reach_1e13(phi, nmod, k):
    dist = "scaled" if phi else "uniform"
    A = _dense(dist, 40, k, 50 + phi, phi)
    B = _dense(dist, k, 30, 51 + phi, phi)
    assert _err_vs_oracle(A, B, oz.crt_emulated(A, B, nmod)) <= 1e-13


def _mutant_reconstruct_unsigned(residues, nmod):
    M = oz.crt_modulus(nmod)
    shape = residues[0].shape
    X = np.empty(shape, dtype=object)
    wts = [(M // m) * pow((M // m) % m, -1, m) for m in oz.MODULI[:nmod]]
    for idx in np.ndindex(*shape):
        X[idx] = sum(int(r[idx]) * wt for r, wt in zip(residues, wts)) % M   # no signed wrap
    return X


def _mutant_reconstruct_no_inverse(residues, nmod):
    M = oz.crt_modulus(nmod)
    shape = residues[0].shape
    X = np.empty(shape, dtype=object)
    wts = [M // m for m in oz.MODULI[:nmod]]     # the inverse factor of each weight dropped
    for idx in np.ndindex(*shape):
        s = sum(int(r[idx]) * wt for r, wt in zip(residues, wts)) % M
        X[idx] = s - M if s >= M // 2 else s
    return X


def _mutant_to_integers_wide(X, w):
    e = oz.row_exponents(X)
    S = np.ldexp(X, (w + 1 - e)[:, None])       # one bit too many
    out = np.empty(X.shape, dtype=object)
    for idx, v in np.ndenumerate(S):
        out[idx] = int(np.trunc(v))
    return out, e


@pytest.mark.parametrize("name,mutant", [("crt_reconstruct", _mutant_reconstruct_unsigned),
                                         ("crt_reconstruct", _mutant_reconstruct_no_inverse),
                                         ("to_integers", _mutant_to_integers_wide)])
def test_planted_mistakes_in_the_crt_reference_are_caught(monkeypatch, name, mutant):
    monkeypatch.setattr(oz, name, mutant)
    with pytest.raises(AssertionError):
        test_crt_reconstruction_is_the_exact_integer_product(8, 15)

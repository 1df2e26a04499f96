"""Helpers shared by the GPU tests: device copies, oracle references, error metrics.

Inputs come from `synth` (seeded, host side); expected values come only from
the CPU oracle or from exact properties, never from the HIP path.
"""
from __future__ import annotations

import numpy as np

import oracle
import synth

TOL = 1e-13


def torch_mod():
    import torch
    return torch


def to_dev(x: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(x).to("cuda")


def run_mdg(p, alpha, beta, variant=-1, C=None):
    """Run the HIP path on problem p (synth.problem dict); returns the host copy of C."""
    import paper_1609_00076_amd as mdg
    torch = torch_mod()
    dA, dB = to_dev(p["A"]), to_dev(p["B"])
    dC = to_dev(p["C"] if C is None else C)
    st = mdg.mdg_dgemm_ex(variant, p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha,
                          dA, p["lda"], dB, p["ldb"], beta, dC, p["ldc"])
    assert st == 0, (f"mdg_dgemm_ex returned {st}: {mdg.mdg_status_string(st)} "
                     f"(hipError_t {mdg.mdg_last_hip_error()})")
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def run_oracle(p, alpha, beta, C=None):
    """(Cref, D): the oracle's C and its error denominator, both flat column-major."""
    C0 = p["C"] if C is None else C
    ref = C0.copy()
    assert oracle.dgemm(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, p["A"],
                        p["lda"], p["B"], p["ldb"], beta, ref, p["ldc"]) == 0
    D = np.zeros(max(1, p["m"] * p["n"]))
    assert oracle.absden(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, p["A"],
                         p["lda"], p["B"], p["ldb"], beta, C0, p["ldc"], D, max(1, p["m"])) == 0
    return ref, D[: p["m"] * p["n"]]


def logical(x, m, n, ld):
    return synth.view2d(x, m, n, ld)


def rel_err(got, ref, D):
    """max |got - ref| / D over entries (D = 0 entries must match exactly)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    D = np.asarray(D, dtype=np.float64).ravel()
    diff = np.abs(got - ref)
    zero = D == 0
    if np.any(zero & (diff != 0)):
        return np.inf
    if got.size == 0:
        return 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(zero, 0.0, diff / np.where(zero, 1.0, D))
    if np.any(np.isnan(r)):
        return np.inf
    return float(r.max())


def same_bits(x, y):
    """Bitwise equality except -0 == +0 and NaN == NaN."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return bool(np.all((np.isnan(x) & np.isnan(y)) | (x == y)))


def padding_untouched(C, p):
    m, n, ldc = p["m"], p["n"], p["ldc"]
    if ldc == m or n == 0:
        return True
    return bool(np.all(C.view(np.uint64).reshape(n, ldc)[:, m:] == synth.PAD_C_BITS))


def check_parity(p, alpha, beta, variant=-1, exact=False, C=None):
    """Run both sides; assert bit-exact (exact=True) or within TOL, and padding untouched."""
    got = run_mdg(p, alpha, beta, variant, C)
    ref, D = run_oracle(p, alpha, beta, C)
    m, n, ldc = p["m"], p["n"], p["ldc"]
    g = logical(got, m, n, ldc)
    r = logical(ref, m, n, ldc)
    tag = f"{p['transa']}{p['transb']} m={m} n={n} k={p['k']} variant={variant}"
    assert padding_untouched(got, p), f"C padding rows written: {tag}"
    if exact:
        assert same_bits(g, r), f"not bit-exact: {tag}"
    else:
        e = rel_err(g.T, r.T, D.reshape(n, m) if m * n else D)
        assert e <= TOL, f"error {e:.3e} > {TOL}: {tag}"
    return got


def sample_indices(size: int, count: int, seed: int):
    """Sorted unique indices: edges, tile boundaries and seeded random ones."""
    fixed = [0, 1, 15, 16, 63, 64, 127, 128, 129, 255, 256, size // 2, size - 2, size - 1]
    g = synth.rng(seed)
    rnd = g.integers(0, size, count).tolist() if size > 0 else []
    return np.array(sorted({i for i in fixed + rnd if 0 <= i < size}), dtype=np.int64)


def _op_dense(x, trans, rows_op, cols_op, ld):
    r, c = synth.stored_dims(trans, rows_op, cols_op)
    v = synth.view2d(x, r, c, ld)
    return v.T if synth.is_trans(trans) else v


def sampled_reference(p, alpha, beta, R, S):
    """Oracle values of full rows R and full columns S of C, with their denominators.

    Only data movement happens here: the needed rows of op(A) and columns of op(B)
    are copied out (as k-contiguous storage, so the oracle's dot products walk
    memory in order) and the oracle evaluates the same definition on them; the
    products and their order per entry are the same as on the whole problem.
    Returns (ref_rows |R| x n, D_rows, ref_cols m x |S|, D_cols) as 2-D arrays.
    """
    ta, tb, m, n, k = p["transa"], p["transb"], p["m"], p["n"], p["k"]
    opa = _op_dense(p["A"], ta, m, k, p["lda"])
    opb = _op_dense(p["B"], tb, k, n, p["ldb"])
    C0 = logical(p["C"], m, n, p["ldc"])
    out = []
    # rows R: op(A)[R, :] stored k x |R| (transposed), op(B) stored k x n
    ar = np.ascontiguousarray(opa[R, :]).reshape(-1)
    if synth.is_trans(tb):
        bn, ldbn = np.ascontiguousarray(opb.T).reshape(-1), max(1, k)
    else:
        bn, ldbn = p["B"], p["ldb"]
    c0r = np.asfortranarray(C0[R, :]).reshape(-1, order="F")
    for fn_abs in (False, True):
        nr = len(R)
        if fn_abs:
            D = np.zeros(nr * n)
            assert oracle.absden("T", "N", nr, n, k, alpha, ar, max(1, k), bn, ldbn, beta, c0r,
                                 max(1, nr), D, max(1, nr)) == 0
            out.append(D.reshape(n, nr).T)
        else:
            c = c0r.copy()
            assert oracle.dgemm("T", "N", nr, n, k, alpha, ar, max(1, k), bn, ldbn, beta, c,
                                max(1, nr)) == 0
            out.append(c.reshape(n, nr).T)
    # columns S: op(A) stored k x m (transposed), op(B)[:, S] stored k x |S|
    if synth.is_trans(ta):
        at, ldat = p["A"], p["lda"]
    else:
        at, ldat = np.ascontiguousarray(opa).reshape(-1), max(1, k)
    bs = np.asfortranarray(opb[:, S]).reshape(-1, order="F")
    c0s = np.asfortranarray(C0[:, S]).reshape(-1, order="F")
    ns = len(S)
    c = c0s.copy()
    assert oracle.dgemm("T", "N", m, ns, k, alpha, at, ldat, bs, max(1, k), beta, c, max(1, m)) == 0
    out.append(c.reshape(ns, m).T)
    D = np.zeros(m * ns)
    assert oracle.absden("T", "N", m, ns, k, alpha, at, ldat, bs, max(1, k), beta, c0s, max(1, m),
                         D, max(1, m)) == 0
    out.append(D.reshape(ns, m).T)
    return out[0], out[1], out[2], out[3]

"""GPU test of the no-allocation split entry point (mdg_dgemm_split_noalloc).

It runs on the library's static scratch array instead of a caller's workspace, with the same
kernels, so its result must equal mdg_dgemm_split's bit for bit. Two calls in a row on one stream,
the second smaller than the first, check that nothing left in the shared array by the first call
leaks into the second (the exponent arrays are cleared by a kernel at the start of each call).
Both results are also checked against the CPU oracle at 1e-13 of D. A problem whose workspace would
exceed the array is refused on the host with MDG_ERR_SCRATCH, leaving C untouched.
"""
import numpy as np
import pytest

import synth
from gpu_util import TOL, logical, rel_err, run_oracle, same_bits

pytestmark = pytest.mark.gpu

# (transa, transb, m, n, k, nslices, phi): the second case is smaller than the first in every
# dimension and in its workspace, so stale bytes of the first call would show in it.
CASES = [("N", "T", 700, 520, 900, 8, 8), ("T", "N", 300, 200, 250, 7, 0)]


def _problem(i, ta, tb, m, n, k, phi):
    dist = "scaled" if phi else "uniform"
    return synth.problem(50, i, ta, tb, m, n, k, ld_rule=lambda r: r + 3, dist=dist, phi=phi)


def _split_with_workspace(p, alpha, beta, S):
    import paper_1609_00076_amd as mdg
    import torch
    dA, dB, dC = (torch.from_numpy(p[x]).cuda() for x in "ABC")
    ws_bytes = mdg.mdg_dgemm_split_workspace_size(p["m"], p["n"], p["k"], S)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    st = mdg.mdg_dgemm_split(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha, dA,
                             p["lda"], dB, p["ldb"], beta, dC, p["ldc"], S, ws, ws_bytes)
    assert st == 0, mdg.mdg_status_string(st)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    import paper_1609_00076_amd as mdg
    import torch
    probs = [(_problem(i, *c[:5], c[6]), c[5]) for i, c in enumerate(CASES)]
    devs = [tuple(torch.from_numpy(p[x]).cuda() for x in "ABC") for p, _ in probs]
    alpha, beta = 1.25, -0.5
    # both calls back to back on the current stream, then one synchronisation
    for (p, S), (dA, dB, dC) in zip(probs, devs):
        need = mdg.mdg_dgemm_split_workspace_size(p["m"], p["n"], p["k"], S)
        assert 0 < need <= mdg.mdg_dgemm_split_noalloc_max_bytes()
        st = mdg.mdg_dgemm_split_noalloc(p["transa"], p["transb"], p["m"], p["n"], p["k"], alpha,
                                         dA, p["lda"], dB, p["ldb"], beta, dC, p["ldc"], S)
        assert st == 0, mdg.mdg_status_string(st)
    torch.cuda.synchronize()
    for (p, S), (_, _, dC) in zip(probs, devs):
        got = dC.cpu().numpy()
        want = _split_with_workspace(p, alpha, beta, S)
        tag = f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']} S={S}"
        assert same_bits(got, want), f"no-alloc result differs from the workspace call: {tag}"
        ref, D = run_oracle(p, alpha, beta)
        m, n, ldc = p["m"], p["n"], p["ldc"]
        err = rel_err(logical(got, m, n, ldc).T, logical(ref, m, n, ldc).T, D)
        assert err <= TOL, f"error {err:.3e} against the oracle: {tag}"
        pad = got.view(np.uint64).reshape(n, ldc)[:, m:]
        assert np.all(pad == synth.PAD_C_BITS), f"C padding written: {tag}"


def test_noalloc_refuses_problems_beyond_the_scratch_array():
    import paper_1609_00076_amd as mdg
    import torch
    cap = mdg.mdg_dgemm_split_noalloc_max_bytes()
    m = n = k = 4096
    assert mdg.mdg_dgemm_split_workspace_size(m, n, k, 8) > cap
    A = torch.zeros(m * k, dtype=torch.float64, device="cuda")
    B = torch.zeros(k * n, dtype=torch.float64, device="cuda")
    C = torch.full((m * n,), 3.0, dtype=torch.float64, device="cuda")
    st = mdg.mdg_dgemm_split_noalloc("N", "N", m, n, k, 1.0, A, m, B, k, 0.0, C, m, 8)
    assert st == mdg.MDG_ERR_SCRATCH
    torch.cuda.synchronize()
    assert bool((C == 3.0).all()), "a refused call must leave C untouched"

"""GPU tests of the continuous-batching server.

* Every kept request's result matches the CPU oracle on its own inputs (1e-13 relative to D),
  native and split-precision alike, and is bitwise the result of serving that request alone.
* Under a small HBM budget a burst of requests is admitted as memory frees up: all complete, the
  budget is never exceeded, and later requests wait for admission.
"""
import copy

import numpy as np
import pytest

import oracle
from gpu_util import TOL, rel_err, same_bits, sample_indices, sampled_reference

pytestmark = pytest.mark.gpu


def _oracle_check(req, kept):
    lda = max(1, req.stored("A")[0])
    ldb = max(1, req.stored("B")[0])
    ldc = max(1, req.m)
    A, B, C0 = (kept[x].cpu().numpy() for x in "ABC")
    ref = C0.copy()
    assert oracle.dgemm(req.transa, req.transb, req.m, req.n, req.k, req.alpha, A, lda, B, ldb,
                        req.beta, ref, ldc) == 0
    D = np.zeros(req.m * req.n)
    assert oracle.absden(req.transa, req.transb, req.m, req.n, req.k, req.alpha, A, lda, B, ldb,
                         req.beta, C0, ldc, D, req.m) == 0
    got = kept["result"].numpy()
    return rel_err(got, ref, D)


def test_served_results_match_oracle_and_alone():
    from paper_1609_00076_amd import serve
    reqs = serve.make_stream(2000, 0.12, seed=11, lo=32, hi=700)
    rng = np.random.default_rng(3)
    keep = set(int(i) for i in rng.choice(len(reqs), size=min(30, len(reqs)), replace=False))
    keep |= {r.rid for r in reqs if r.kind == "split"}
    keep |= {r.rid for r in reqs if serve.route_of(r) == "single"}
    srv = serve.Server(keep=keep)
    stats = srv.run(reqs)
    s = stats.summary()
    assert s["requests"] == len(reqs)
    assert s["grouped_requests"] > 0 and s["split_requests"] > 0
    assert any(serve.route_of(r) == "single" for r in reqs)
    mixed = srv.kept
    for rid in sorted(keep):
        req = reqs[rid]
        err = _oracle_check(req, mixed[rid])
        assert err <= TOL, f"request {rid} ({req.kind}, {serve.route_of(req)}): error {err:.2e}"
        # the same request served alone
        import copy
        solo = copy.copy(req)
        solo.arrival = 0.0
        srv1 = serve.Server(keep={rid})
        srv1.run([solo])
        assert same_bits(srv1.kept[rid]["result"].numpy(), mixed[rid]["result"].numpy()), rid


def test_budget_limits_admission():
    from paper_1609_00076_amd import serve
    reqs = serve.make_stream(20000, 0.01, seed=12, lo=64, hi=256, split_fraction=0.0)
    for r in reqs:
        r.arrival = 0.0  # a burst
    srv = serve.Server(keep=None)
    biggest = max(srv.request_bytes(r) for r in reqs)
    srv.budget_bytes = 3 * biggest
    stats = srv.run(reqs)
    s = stats.summary()
    assert s["requests"] == len(reqs) > 50
    assert stats.peak_bytes <= srv.budget_bytes
    assert s["scheduler_passes"] > 1  # admission happened in several passes as memory freed
    waited = [r for r in stats.records if r.admitted > 1e-3]
    assert waited


def _as_problem(req, kept):
    return dict(transa=req.transa, transb=req.transb, m=req.m, n=req.n, k=req.k,
                A=kept["A"].cpu().numpy(), lda=max(1, req.stored("A")[0]),
                B=kept["B"].cpu().numpy(), ldb=max(1, req.stored("B")[0]),
                C=kept["C"].cpu().numpy(), ldc=max(1, req.m))


def test_served_stream_full_shape_range():
    """The served workload's shape range: m, n, k log-uniform in [32, 4096], 20% split requests at
    phi = 8 (9 slices), 80% native. Every kept request is checked against the oracle at 1e-13 of D
    (in full up to 2^27 multiply-adds, else on sampled full rows and columns), and is bitwise the
    same when served alone."""
    from paper_1609_00076_amd import serve
    reqs = serve.make_stream(2000, 0.05, seed=21, lo=32, hi=4096, split_fraction=0.2, phi=8)
    assert len(reqs) >= 60
    big = [r for r in reqs if max(r.m, r.n, r.k) > 2048]
    assert big, "the stream should hold requests near the top of the range"
    keep = {r.rid for r in reqs}
    srv = serve.Server(keep=keep)
    s = srv.run(reqs).summary()
    assert s["requests"] == len(reqs) and s["split_requests"] > 0 and s["grouped_requests"] > 0
    mixed = srv.kept
    print(f"[serve] {len(reqs)} requests served; checking each", flush=True)
    for r in reqs:
        kept = mixed[r.rid]
        tag = f"request {r.rid} ({r.kind}, {serve.route_of(r)}, {r.transa}{r.transb} {r.m}x{r.n}x{r.k})"
        if r.m * r.n * r.k <= (1 << 27):
            err = _oracle_check(r, kept)
        else:
            p = _as_problem(r, kept)
            R = sample_indices(r.m, 6, r.seed % 100000)
            S = sample_indices(r.n, 6, r.seed % 100000 + 1)
            ref_r, d_r, ref_c, d_c = sampled_reference(p, r.alpha, r.beta, R, S)
            got = kept["result"].numpy().reshape(r.n, r.m).T
            err = max(rel_err(got[R, :], ref_r, d_r), rel_err(got[:, S], ref_c, d_c))
        assert err <= TOL, f"{tag}: error {err:.2e}"
        solo = copy.copy(r)
        solo.arrival = 0.0
        srv1 = serve.Server(keep={r.rid})
        srv1.run([solo])
        assert same_bits(srv1.kept[r.rid]["result"].numpy(), kept["result"].numpy()), tag
        del mixed[r.rid]
    print(f"[serve] all {len(reqs)} requests match the oracle and their solo runs", flush=True)

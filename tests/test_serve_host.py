"""Host-side parts of the server on the CPU: request stream, admission, statistics."""
import math

import numpy as np
import pytest

from paper_1609_00076_amd import serve


def test_stream_is_seeded_poisson_with_the_requested_mix():
    a = serve.make_stream(2000, 5.0, seed=7)
    b = serve.make_stream(2000, 5.0, seed=7)
    assert [(r.arrival, r.m, r.n, r.k, r.kind, r.seed) for r in a] == \
        [(r.arrival, r.m, r.n, r.k, r.kind, r.seed) for r in b]
    assert abs(len(a) - 10000) < 4 * math.sqrt(10000)
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 2000) < 0.05 / 2000
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.05  # exponential: cv = 1
    dims = np.array([(r.m, r.n, r.k) for r in a])
    assert dims.min() >= 32 and dims.max() <= 4096
    assert abs(np.mean(np.log(dims)) - (math.log(32) + math.log(4097)) / 2) < 0.05
    split = [r for r in a if r.kind == "split"]
    assert abs(len(split) / len(a) - 0.2) < 0.02 and all(r.phi == 8 for r in split)
    assert {r.transa for r in a} == {"N", "T"}


def test_admission_is_fifo_under_the_budget():
    q = serve.AdmissionQueue(100)
    reqs = [serve.Request(i, 0.0, "native", "N", "N", 1, 1, 1, 1.0, 0.0, i) for i in range(4)]
    for r, nb in zip(reqs, (60, 30, 50, 10)):
        q.offer(r, nb)
    first = q.admit()
    assert [r.rid for r, _ in first] == [0, 1]       # 60 + 30 fit; 50 must wait
    assert q.admit() == []                            # no overtaking: 10 waits behind 50
    q.release(60)
    assert [r.rid for r, _ in q.admit()] == [2, 3]
    assert q.peak_used == 90 and q.free == 10
    with pytest.raises(ValueError):
        q.offer(reqs[0], 101)


def test_percentiles_and_summary():
    assert serve.percentile([5, 1, 3, 2, 4], 50) == 3
    assert serve.percentile(list(range(1, 101)), 99) == 99
    st = serve.RunStats(records=[serve.Record(i, "native", "single", 2e12, 0.0, 0.0, (i + 1) * 1e-3)
                                 for i in range(100)], wall=2.0)
    s = st.summary()
    assert s["requests"] == 100 and s["p50_ms"] == 50.0 and s["p99_ms"] == 99.0
    assert s["aggregate_tflops"] == 100.0


def test_routing_depends_only_on_the_request():
    r = serve.Request(0, 0.0, "native", "N", "T", 512, 100, 4000, 1.0, 1.0, 1)
    assert serve.route_of(r) == "grouped"
    r.n = 513
    assert serve.route_of(r) == "single"
    r.kind = "split"
    assert serve.route_of(r) == "split"

"""Continuous-batching server for dgemm requests on one GPU.

Requests arrive over time (a seeded Poisson stream), each one GEMM C := alpha*op(A)*op(B) + beta*C
computed either natively in FP64 or by the split-precision path (INT8 products recombined by the
Chinese remainder theorem). The server loop:

1. moves requests whose arrival time has passed into a FIFO admission queue;
2. admits from the head of the queue while the request's device bytes (operands, plus the
   workspace of a split request) fit in the remaining HBM budget; an admitted request's operands
   are materialised on the device from its own seed, so no host data crosses PCIe;
3. launches everything admitted in this pass: requests with max(m, n) <= `group_max_dim` and
   native arithmetic go into one grouped persistent launch, larger native ones get their own
   launch, split ones run the split path; launches rotate over several streams, so work admitted
   while earlier work is still on the GPU overlaps with it;
4. polls completion events; a finished request releases its bytes to the budget and records its
   latency (arrival to observed completion).

The routing of a request (grouped or single launch, tile class, modulus count) depends only on the
request itself, so its result is the same alone and in any mix.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

GROUP_MAX_DIM = 512
GROUP_THRESHOLD = 40   # grouped tile class 1 (32x32) when min(m, n) < this
# Split requests run the Chinese-remainder split (one INT8 product per modulus). Moduli per
# exponent spread phi for requests with k down to 32: at phi = 8 a row of 32 entries needs 16 to keep
# max |C - Cref| / (|A||B|)_ij under 1e-13 (15 suffice at k = 2048 and beyond).
SPLIT_MODULI = {0: 14, 8: 16}


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the stream
    kind: str               # "native" or "split"
    transa: str
    transb: str
    m: int
    n: int
    k: int
    alpha: float
    beta: float
    seed: int
    phi: int = 0

    @property
    def flops(self) -> float:
        return 2.0 * self.m * self.n * self.k

    def stored(self, which):
        if which == "A":
            return (self.k, self.m) if self.transa == "T" else (self.m, self.k)
        if which == "B":
            return (self.n, self.k) if self.transb == "T" else (self.k, self.n)
        return (self.m, self.n)

    def operand_bytes(self) -> int:
        return sum(8 * r * c for r, c in (self.stored(x) for x in "ABC"))


def make_stream(rate: float, duration: float, seed: int, lo: int = 32, hi: int = 4096,
                split_fraction: float = 0.2, phi: int = 8) -> list:
    """Seeded Poisson arrivals at `rate` per second for `duration` seconds; shapes log-uniform
    integers in [lo, hi], transposes iid, alpha and beta ~ U[-1, 1), a `split_fraction` share of
    split-precision requests with exponent spread phi."""
    g = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    t = 0.0
    rid = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        m, n, k = (int(x) for x in np.clip(np.floor(np.exp(g.uniform(math.log(lo), math.log(hi + 1), 3))), lo, hi))
        kind = "split" if g.uniform() < split_fraction else "native"
        reqs.append(Request(rid, t, kind, "NT"[g.integers(2)], "NT"[g.integers(2)], m, n, k,
                            float(g.uniform(-1, 1)), float(g.uniform(-1, 1)),
                            int(g.integers(1 << 62)), phi if kind == "split" else 0))
        rid += 1
    return reqs


class AdmissionQueue:
    """FIFO admission under a byte budget (no request overtakes an earlier one)."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.free = int(budget_bytes)
        self.queue = deque()
        self.peak_used = 0

    def offer(self, req, nbytes: int):
        if nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {nbytes} bytes, more than the whole budget")
        self.queue.append((req, int(nbytes)))

    def admit(self):
        out = []
        while self.queue and self.queue[0][1] <= self.free:
            req, nbytes = self.queue.popleft()
            self.free -= nbytes
            out.append((req, nbytes))
        self.peak_used = max(self.peak_used, self.budget - self.free)
        return out

    def release(self, nbytes: int):
        self.free += int(nbytes)
        assert self.free <= self.budget


def percentile(values, q):
    if not values:
        return float("nan")
    v = sorted(values)
    idx = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[idx]


@dataclass
class Record:
    rid: int
    kind: str
    route: str
    flops: float
    arrival: float
    admitted: float
    completed: float

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@dataclass
class RunStats:
    records: list = field(default_factory=list)
    wall: float = 0.0
    peak_bytes: int = 0
    passes: int = 0
    grouped_launches: int = 0

    def summary(self):
        lat = [r.latency for r in self.records]
        flops = sum(r.flops for r in self.records)
        return {
            "requests": len(self.records),
            "split_requests": sum(r.kind == "split" for r in self.records),
            "grouped_requests": sum(r.route == "grouped" for r in self.records),
            "p50_ms": round(1e3 * percentile(lat, 50), 4),
            "p99_ms": round(1e3 * percentile(lat, 99), 4),
            "mean_ms": round(1e3 * (sum(lat) / len(lat)), 4) if lat else float("nan"),
            "aggregate_tflops": round(flops / self.wall / 1e12, 4) if self.wall else float("nan"),
            "offered_tflop": round(flops / 1e12, 4),
            "wall_s": round(self.wall, 3),
            "peak_budget_bytes": self.peak_bytes,
            "scheduler_passes": self.passes,
            "grouped_launches": self.grouped_launches,
        }


def route_of(req) -> str:
    if req.kind == "split":
        return "split"
    return "grouped" if max(req.m, req.n) <= GROUP_MAX_DIM else "single"


class Server:
    """One-GPU continuous-batching server (torch supplies memory, streams and the seeded fills)."""

    def __init__(self, budget_bytes=64 << 30, streams=4, keep=None):
        import torch

        import paper_1609_00076_amd as mdg
        self.torch = torch
        self.mdg = mdg
        self.budget_bytes = budget_bytes
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.next_stream = 0
        self.gen = torch.Generator(device="cuda")
        self.keep = keep  # set of request ids whose inputs and result are copied back, or None

    # -- per-request device work ---------------------------------------------------------------
    def request_bytes(self, req):
        nb = req.operand_bytes()
        if req.kind == "split":
            nb += self.mdg.mdg_dgemm_crt_workspace_size(req.m, req.n, req.k,
                                                        SPLIT_MODULI[req.phi])
        return nb

    def _fill(self, t, req):
        torch = self.torch
        t.uniform_(-1.0, 1.0, generator=self.gen)
        if req.phi:
            e = torch.randint(-req.phi, req.phi + 1, t.shape, generator=self.gen, device="cuda",
                              dtype=torch.int32)
            t.copy_(torch.ldexp(t, e))

    def materialize(self, req, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            self.gen.manual_seed(req.seed)
            ops = {}
            for x in "ABC":
                r, c = req.stored(x)
                t = torch.empty(max(1, r * c), dtype=torch.float64, device="cuda")
                self._fill(t, req)
                ops[x] = t
            if req.kind == "split":
                nb = self.mdg.mdg_dgemm_crt_workspace_size(req.m, req.n, req.k,
                                                           SPLIT_MODULI[req.phi])
                ops["W"] = torch.empty(max(256, nb), dtype=torch.uint8, device="cuda")
        return ops

    def gemm_args(self, req, ops):
        lda = max(1, req.stored("A")[0])
        ldb = max(1, req.stored("B")[0])
        ldc = max(1, req.m)
        return (req.transa, req.transb, req.m, req.n, req.k, req.alpha, ops["A"], lda, ops["B"],
                ldb, req.beta, ops["C"], ldc)

    def launch_single(self, req, ops, stream):
        args = self.gemm_args(req, ops)
        if req.kind == "split":
            st = self.mdg.mdg_dgemm_crt(*args, SPLIT_MODULI[req.phi], ops["W"], ops["W"].numel(),
                                        stream=stream)
        else:
            st = self.mdg.mdg_dgemm(*args, stream=stream)
        if st:
            raise self.mdg.MdgError(st)

    def launch_group(self, items, stream):
        from .grouped import GroupedPlan
        gemms, classes = [], []
        for req, ops in items:
            a = self.gemm_args(req, ops)
            gemms.append(dict(transa=a[0], transb=a[1], m=a[2], n=a[3], k=a[4], alpha=a[5],
                              A=a[6], lda=a[7], B=a[8], ldb=a[9], beta=a[10], C=a[11], ldc=a[12]))
            classes.append(1 if min(req.m, req.n) < GROUP_THRESHOLD else 0)
        with self.torch.cuda.stream(stream):
            plan = GroupedPlan(gemms, classes, self.mdg.MDG_SCHEDULE_LPT)
            plan.launch(0, stream)
        return plan

    # -- the loop -----------------------------------------------------------------------------
    def run(self, requests):
        """Serve `requests` in real time (arrival times are seconds from the call); returns
        RunStats. Kept requests' inputs and results are left in self.kept."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        queue = AdmissionQueue(self.budget_bytes)
        inflight = []   # (event, [(req, nbytes, ops, admitted_t)], keepalive)
        stats = RunStats()
        kept = {}
        pending = deque(reqs)
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        while pending or queue.queue or inflight:
            t = now()
            while pending and pending[0].arrival <= t:
                r = pending.popleft()
                queue.offer(r, self.request_bytes(r))
            admitted = queue.admit()
            if admitted:
                stats.passes += 1
                tadm = now()
                groups, singles = [], []
                for req, nb in admitted:
                    stream = self.streams[self.next_stream % len(self.streams)]
                    self.next_stream += 1
                    ops = self.materialize(req, stream)
                    if req.rid in (self.keep or ()):
                        with torch.cuda.stream(stream):  # after the fills, before the GEMM
                            kept[req.rid] = {x: ops[x].clone() for x in "ABC"}
                    (groups if route_of(req) == "grouped" else singles).append((req, nb, ops, stream))
                if groups:
                    # the grouped launch waits for every member's materialisation stream
                    gstream = self.streams[self.next_stream % len(self.streams)]
                    self.next_stream += 1
                    for s in {id(s): s for _, _, _, s in groups}.values():
                        gstream.wait_stream(s)
                    plan = self.launch_group([(r, o) for r, _, o, _ in groups], gstream)
                    stats.grouped_launches += 1
                    ev = torch.cuda.Event()
                    ev.record(gstream)
                    inflight.append((ev, [(r, nb, o, tadm) for r, nb, o, _ in groups], plan))
                for req, nb, ops, stream in singles:
                    self.launch_single(req, ops, stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                    inflight.append((ev, [(req, nb, ops, tadm)], None))
            still = []
            for ev, members, keep in inflight:
                if ev.query():
                    tdone = now()
                    for req, nb, ops, tadm in members:
                        if req.rid in kept:
                            kept[req.rid]["result"] = ops["C"].cpu()
                        stats.records.append(Record(req.rid, req.kind, route_of(req), req.flops,
                                                    req.arrival, tadm, tdone))
                        queue.release(nb)
                else:
                    still.append((ev, members, keep))
            inflight = still
            if not admitted and not still and pending:
                gap = pending[0].arrival - now()
                if gap > 2e-4:
                    time.sleep(gap - 1e-4)
        stats.wall = now()
        stats.peak_bytes = queue.peak_used
        self.kept = kept
        return stats

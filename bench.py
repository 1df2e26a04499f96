#!/usr/bin/env python3
"""FP64 GEMM benchmark on one MI355X: native dgemm sweep through the C ABI.

One step = one pass over the sweep workload: the four (transa, transb) cases of
square m = n = k in {1024, 2048, 4096, 4099, 8192, 16384} and the skinny
m = n = 8192, k = 64 (28 GEMMs), ld = stored rows rounded up to a multiple of 8,
alpha = beta = 1, Uniform[-1,1] entries drawn by the seeded generator and
resident in HBM before timing starts. value = total 2mnk flops / timed seconds.

Prints ONE JSON line (rank 0). Only one GPU is supported: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 GEMM TFLOP/s (% of MFMA peak), native vs split-precision at err<=1e-13"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
SQUARES = [1024, 2048, 4096, 4099, 8192, 16384]
SKINNY = (8192, 8192, 64)
TRANS = ["NN", "NT", "TN", "TT"]
SOURCE = os.path.join(ROOT, "paper_1609_00076_amd", "csrc", "mdg_dgemm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
BLAS3_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blas3_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    return hashlib.sha256(open(SOURCE, "rb").read()).hexdigest()[:16]


def build_problems(torch, shapes_filter=None):
    """Seeded host operands for the sweep and their device copies (square sizes share A, B, C
    across the four transpose cases). Returns a list of problems with host arrays hA, hB, hC and
    device tensors A, B, C."""
    import synth
    probs = []
    for size in SQUARES:
        if shapes_filter and size not in shapes_filter:
            continue
        ld = synth.ld_round8(size)
        hA = synth.matrix(synth.seed_for(2, 100, 0), size, size, ld)
        hB = synth.matrix(synth.seed_for(2, 100, 1), size, size, ld)
        hC = synth.matrix(synth.seed_for(2, 100, 2), size, size, ld, pad=synth.pad_c_value())
        A, B, C = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
        for tr in TRANS:
            probs.append(dict(transa=tr[0], transb=tr[1], m=size, n=size, k=size, A=A, lda=ld,
                              B=B, ldb=ld, C=C, ldc=ld, hA=hA, hB=hB, hC=hC))
        log(f"[bench] operands for {size}^3 resident")
    if not shapes_filter or "skinny" in shapes_filter:
        m, n, k = SKINNY
        ldc = synth.ld_round8(m)
        hC = synth.matrix(synth.seed_for(2, 101, 2), m, n, ldc, pad=synth.pad_c_value())
        C = torch.from_numpy(hC).cuda()
        for t, tr in enumerate(TRANS):
            ra, ca = synth.stored_dims(tr[0], m, k)
            rb, cb = synth.stored_dims(tr[1], k, n)
            lda, ldb = synth.ld_round8(ra), synth.ld_round8(rb)
            hA = synth.matrix(synth.seed_for(2, 110 + t, 0), ra, ca, lda)
            hB = synth.matrix(synth.seed_for(2, 110 + t, 1), rb, cb, ldb)
            A, B = torch.from_numpy(hA).cuda(), torch.from_numpy(hB).cuda()
            probs.append(dict(transa=tr[0], transb=tr[1], m=m, n=n, k=k, A=A, lda=lda, B=B,
                              ldb=ldb, C=C, ldc=ldc, hA=hA, hB=hB, hC=hC))
        log("[bench] operands for 8192x8192x64 resident")
    return probs


def out_workload(probs):
    return sorted({f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']}" for p in probs})


def flops(p):
    return 2.0 * p["m"] * p["n"] * p["k"]


def hbm_bytes(p, beta=1.0):
    """Algorithmic bytes: read op(A), op(B) once, read C if beta != 0, write C once."""
    m, n, k = p["m"], p["n"], p["k"]
    return 8.0 * (m * k + k * n + m * n * (beta != 0.0) + m * n)


def kernel_key(mdg, p, variant=-1):
    v = variant if variant >= 0 else \
        mdg.mdg_select_variant(p["transa"], p["transb"], p["m"], p["n"], p["k"], 1.0, 1.0)
    return f"{mdg.mdg_variant_name(v)}[{p['transa']}{p['transb']}]"


def run_step(mdg, probs, events=None, variant=-1):
    for i, p in enumerate(probs):
        if events is not None:
            events[i][0].record()
        st = mdg.mdg_dgemm_ex(variant, p["transa"], p["transb"], p["m"], p["n"], p["k"], 1.0,
                              p["A"], p["lda"], p["B"], p["ldb"], 1.0, p["C"], p["ldc"])
        if st:
            raise RuntimeError(f"mdg_dgemm failed: {mdg.mdg_status_string(st)}")
        if events is not None:
            events[i][1].record()


def cpu_baseline(probs, budget_s: float, threads: int = 0):
    """Time the CPU oracle on blocks of the sweep problems, on the host copies of the inputs.

    Each problem gets an equal share of the budget. Within it the oracle computes
    consecutive r x c blocks of C (c = one column per thread, r starting at 16 rows and
    doubling while a call takes under a quarter of the share), walking down the leading
    columns, on the problem's own arrays with pointer offsets (no data movement; the
    results go to a scratch C). threads = 0 uses every host thread OpenMP offers.
    Returns (TFLOP/s, threads, description).
    """
    import numpy as np

    import oracle
    oracle.set_threads(threads)
    threads = oracle.get_threads()
    share = budget_s / len(probs)
    total_flops, total_t, entries = 0.0, 0.0, 0
    for p in probs:
        m, n, k = p["m"], p["n"], p["k"]
        ta, tb, lda, ldb = p["transa"], p["transb"], p["lda"], p["ldb"]
        hA, hB = p["hA"], p["hB"]
        C = np.zeros(m * threads)
        spent, i0, j0, r = 0.0, 0, 0, min(16, m)
        while spent < share and j0 < n:
            rr, c = min(r, m - i0), min(threads, n - j0)
            aoff = i0 if ta == "N" else i0 * lda   # rows i0.. of op(A)
            boff = j0 * ldb if tb == "N" else j0   # columns j0.. of op(B)
            t0 = time.perf_counter()
            st = oracle.dgemm(ta, tb, rr, c, k, 1.0, hA[aoff:], lda, hB[boff:], ldb, 1.0, C, m)
            dt = time.perf_counter() - t0
            assert st == 0
            spent += dt
            total_t += dt
            total_flops += 2.0 * rr * c * k
            entries += rr * c
            i0 += rr
            if i0 >= m:
                i0, j0 = 0, j0 + c
            if dt < share / 4:
                r *= 2
    oracle.set_threads(0)
    desc = (f"oracle on leading blocks of C of each of the {len(probs)} sweep GEMMs "
            f"({entries} entries of C, {total_t:.1f} s, one column per thread per call)")
    return total_flops / total_t / 1e12, threads, desc


SPLIT_CASES = [(0, 7), (8, 8), (32, 10)]  # (phi, nslices) that reach err <= 1e-13
INT8_PEAK_TOPS = 5000.0


def split_workload(args, torch, mdg):
    """Split-precision dgemm (INT8 MFMA slices) against the native FP64 kernel, NN 8192^3."""
    import numpy as np

    import synth
    m = n = k = args.split_size
    results = []
    for phi, S in SPLIT_CASES:
        dist = "scaled" if phi else "uniform"
        p = synth.problem(3, phi, "N", "N", m, n, k, ld_rule=synth.ld_round8, dist=dist, phi=phi)
        dA, dB, dC0 = (torch.from_numpy(p[x]).cuda() for x in "ABC")
        ws_bytes = mdg.mdg_dgemm_split_workspace_size(m, n, k, S)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        dC = dC0.clone()

        def split_call():
            st = mdg.mdg_dgemm_split("N", "N", m, n, k, 1.0, dA, p["lda"], dB, p["ldb"], 1.0, dC,
                                     p["ldc"], S, ws, ws_bytes)
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))

        def native_call():
            st = mdg.mdg_dgemm("N", "N", m, n, k, 1.0, dA, p["lda"], dB, p["ldb"], 1.0, dC,
                               p["ldc"])
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))

        times = {}
        for name, fn in (("split", split_call), ("native", native_call)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / args.steps
        # Accuracy over the whole of C, on the GPU: one split call and one native call from the
        # original C, and D = |A||B| + |C0| from a native call on absolute values. The native FP64
        # result is within rounding (about 1e-16 D) of the exact one, so this bounds the split
        # error against the exact product to that margin. (The test suite checks the same inputs
        # against the CPU oracle.)
        dC.copy_(dC0)
        split_call()
        c_split = dC.clone()
        dC.copy_(dC0)
        native_call()
        dD = dC0.abs()
        st = mdg.mdg_dgemm("N", "N", m, n, k, 1.0, dA.abs(), p["lda"], dB.abs(), p["ldb"], 1.0, dD,
                           p["ldc"])
        if st:
            raise RuntimeError(mdg.mdg_status_string(st))
        ld = p["ldc"]
        diff = (c_split.view(n, ld)[:, :m] - dC.view(n, ld)[:, :m]).abs()
        den = dD.view(n, ld)[:, :m]
        ratio = torch.where(den > 0, diff / den, torch.where(diff > 0, float("inf"), 0.0))
        err = float(ratio.max())
        del dA, dB, dC, dC0, dD, ws, c_split, diff, den, ratio
        fl = 2.0 * m * n * k
        products = S * (S + 1) // 2
        results.append({
            "phi": phi, "nslices": S, "slice_products": products,
            "split_ms": round(times["split"], 3), "native_ms": round(times["native"], 3),
            "split_tflops_equiv": round(fl / (times["split"] * 1e-3) / 1e12, 2),
            "native_tflops": round(fl / (times["native"] * 1e-3) / 1e12, 2),
            "int8_tops_in_call": round(products * fl / (times["split"] * 1e-3) / 1e12, 1),
            "speedup_vs_native": round(times["native"] / times["split"], 3),
            "max_err_vs_native_fp64": float(f"{err:.3g}"),
        })
        log(f"[bench] split phi={phi} S={S}: {results[-1]}")
    best = max(results, key=lambda r: r["split_tflops_equiv"])
    out = {
        "metric": METRIC + " (split-precision leg)",
        "value": best["split_tflops_equiv"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8 slices, f64 recombination",
        "data": "synthetic: seeded u*2^e, u ~ U[-1,1), e ~ U{-phi..phi}",
        "config": {"workload": f"split-precision dgemm NN {m}x{n}x{k}, ld rounded to 8, alpha=beta=1",
                   "cases": results},
        "roofline": {"bound": "mfma", "peak": INT8_PEAK_TOPS, "unit": "TOP/s (int8)",
                     "achieved": best["int8_tops_in_call"],
                     "frac": round(best["int8_tops_in_call"] / INT8_PEAK_TOPS, 4),
                     "note": "whole call (slicing + fused GEMM) time; the kernel alone is in profiles/"},
    }
    print(json.dumps(out), flush=True)


def grouped_problems(count=2048, lo=16, hi=512, seed_variant=0):
    """Workload of 2048 independent GEMMs: m, n, k log-uniform integers in [lo, hi], transposes
    iid, alpha and beta ~ U[-1, 1), tight leading dimensions, entries U[-1, 1)."""
    import synth
    return synth.grouped_batch(count, lo, hi, seed_variant)


def grouped_workload(args, torch, mdg):
    """2048 uneven GEMMs: one grouped launch replayed from a graph, against per-GEMM launches."""
    from paper_1609_00076_amd import tuner
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = grouped_problems()
    gemms = []
    for p in probs:
        gemms.append(dict(transa=p["transa"], transb=p["transb"], m=p["m"], n=p["n"], k=p["k"],
                          alpha=p["alpha"], beta=p["beta"], lda=p["lda"], ldb=p["ldb"],
                          ldc=p["ldc"], A=torch.from_numpy(p["A"]).cuda(),
                          B=torch.from_numpy(p["B"]).cuda(), C=torch.from_numpy(p["C"]).cuda()))
    torch.cuda.synchronize()
    log(f"[bench] {len(gemms)} GEMMs resident")
    total_flops = sum(2.0 * g["m"] * g["n"] * g["k"] for g in gemms)
    total_bytes = sum(8.0 * (g["m"] * g["k"] + g["k"] * g["n"] + 2 * g["m"] * g["n"]) for g in gemms)
    db = args.tune_db or tuner.DB_PATH
    if args.tune:
        entry = tuner.tune_grouped(gemms, tuner.GROUPED_SIGNATURE, db_path=db, log=log)
        policy = entry["policy"]
    else:
        policy = tuner.best_policy(tuner.GROUPED_SIGNATURE, db_path=db)
    log(f"[bench] policy {policy}")

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    plan = GroupedPlan(gemms, tuner.classes_for(gemms, policy["threshold"]), policy["schedule"])
    eager_grouped = timed(lambda: plan.launch(policy["grid"]), args.steps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.launch(policy["grid"])
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch(policy["grid"])
    graph_ms = timed(graph.replay, args.steps)

    def per_gemm():
        for g in gemms:
            st = mdg.mdg_dgemm(g["transa"], g["transb"], g["m"], g["n"], g["k"], g["alpha"],
                               g["A"], g["lda"], g["B"], g["ldb"], g["beta"], g["C"], g["ldc"])
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))
    separate_ms = timed(per_gemm, max(1, args.steps // 4))
    value = total_flops / (graph_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC + " (grouped-launch leg)",
        "value": round(value, 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded U[-1,1) FP64, shapes log-uniform in [16,512]",
        "config": {"workload": "2048 independent dgemm, m,n,k log-uniform integers in [16,512], "
                               "transposes iid, alpha,beta ~ U[-1,1), tight ld; one grouped "
                               "persistent launch replayed from a graph",
                   "policy": policy, "tiles": plan.num_tiles,
                   "total_flops": total_flops, "algorithmic_bytes": total_bytes},
        "graph_replay_ms": round(graph_ms, 4),
        "eager_grouped_ms": round(eager_grouped, 4),
        "separate_launches_ms": round(separate_ms, 4),
        "speedup_vs_separate": round(separate_ms / graph_ms, 2),
        "roofline": {"bound": "hbm", "achieved": round(total_bytes / (graph_ms * 1e-3) / 1e9, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(total_bytes / (graph_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "mfma_frac": round(value / PEAK_FP64_MFMA_TFLOPS, 4), "traffic": None},
    }
    print(json.dumps(out), flush=True)


def served_workload(args, torch, mdg):
    """Poisson stream of dgemm requests through the continuous-batching server."""
    from paper_1609_00076_amd import serve
    reqs = serve.make_stream(args.rate, args.duration, seed=synth_seed(5), lo=32, hi=4096,
                             split_fraction=0.2, phi=8)
    log(f"[bench] serving {len(reqs)} requests over {args.duration} s")
    warm = serve.make_stream(200, 0.5, seed=synth_seed(5) + 1, lo=32, hi=512)
    srv = serve.Server(budget_bytes=args.budget_gb << 30)
    srv.run(warm)  # compile-free warm-up of allocator and streams
    stats = srv.run(reqs)
    s = stats.summary()
    log(f"[bench] served: {s}")
    out = {
        "metric": METRIC + " (served-stream leg)",
        "value": s["aggregate_tflops"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * s["wall_s"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: operands filled on the device from per-request seeds",
        "config": {"workload": f"Poisson {args.rate:g} req/s for {args.duration:g} s, m,n,k "
                               "log-uniform in [32,4096], transposes iid, 80% native, 20% split "
                               f"(phi=8, {serve.SPLIT_SLICES[8]} slices), HBM budget "
                               f"{args.budget_gb} GB"},
        "served": s,
    }
    print(json.dumps(out), flush=True)


BLAS3_SIZE = 8192


def blas3_cpu_baseline(hA, hT, hB, n, budget_s: float):
    """The oracle's dsyrk, dtrmm and dtrsm on samples of the level-3 problems (host copies):
    dsyrk on the leading n_s x n_s triangle with the full k, dtrmm and dtrsm on the leading c
    columns of B (each column is an independent right-hand side) with the full order n. Sample
    sizes double until each call takes a third of the budget. Returns (TFLOP/s, threads, text)."""
    import numpy as np

    import oracle
    threads = oracle.get_threads()
    share = budget_s / 3
    total_flops, total_t, parts = 0.0, 0.0, []
    ns = 64
    while True:
        C = np.zeros(ns * ns)
        t0 = time.perf_counter()
        assert oracle.dsyrk("L", "N", ns, n, 1.0, hA, n, 0.0, C, ns) == 0
        dt = time.perf_counter() - t0
        if dt >= share / 4 or ns >= n:
            total_flops += float(ns) * (ns + 1) * n
            total_t += dt
            parts.append(f"dsyrk L N {ns}x{ns} k={n} ({dt:.1f} s)")
            break
        ns *= 2
    for name in ("dtrmm", "dtrsm"):
        c = threads
        while True:
            Bs = np.ascontiguousarray(hB[: n * c]).copy()
            t0 = time.perf_counter()
            assert getattr(oracle, name)("L", "L", "N", "N", n, c, 1.0, hT, n, Bs, n) == 0
            dt = time.perf_counter() - t0
            if dt >= share / 4 or c >= n:
                total_flops += float(n) * n * c
                total_t += dt
                parts.append(f"{name} L L N N {n}x{c} ({dt:.1f} s)")
                break
            c *= 2
    return total_flops / total_t / 1e12, threads, "oracle on " + "; ".join(parts)


def blas3_workload(args, torch, mdg):
    """Level-3 operations built on the GEMM, n = 8192: dsyrk (lower, 'N', k = n), dtrmm and
    dtrsm (side L, lower, 'N', non-unit, m = n). One step = the three calls."""
    import synth
    n = BLAS3_SIZE
    hA = synth.matrix(synth.seed_for(64, 0, 0), n, n, n)
    hC = synth.matrix(synth.seed_for(64, 0, 2), n, n, n)
    hT = synth.triangular(synth.seed_for(64, 0, 3), n, n, "L", "uniform")
    hB = synth.matrix(synth.seed_for(64, 0, 1), n, n, n)
    dA, dC, dT, dB = (torch.from_numpy(x).cuda() for x in (hA, hC, hT, hB))
    log("[bench] level-3 operands resident")
    ops = {
        "dsyrk": (lambda: mdg.mdg_dsyrk("L", "N", n, n, 1.0, dA, n, 1.0, dC, n), float(n) * (n + 1) * n),
        "dtrmm": (lambda: mdg.mdg_dtrmm("L", "L", "N", "N", n, n, 1.0, dT, n, dB, n), float(n) * n * n),
        # solving with the matrix that trmm just multiplied in keeps B bounded step after step
        "dtrsm": (lambda: mdg.mdg_dtrsm("L", "L", "N", "N", n, n, 1.0, dT, n, dB, n), float(n) * n * n),
    }

    def step(events=None):
        for i, (name, (fn, _)) in enumerate(ops.items()):
            if events is not None:
                events[i][0].record()
            st = fn()
            if st:
                raise RuntimeError(f"{name}: {mdg.mdg_status_string(st)}")
            if events is not None:
                events[i][1].record()

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {w + 1}/{args.warmup} done")
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in ops] for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        step(ev[s])
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    log(f"[bench] {args.steps} timed level-3 steps done in {total_ms:.1f} ms")
    step_flops = sum(f for _, f in ops.values())
    value = step_flops * args.steps / (total_ms * 1e-3) / 1e12
    by_op = {}
    for i, (name, (_, fl)) in enumerate(ops.items()):
        ms = sorted(ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps))
        med = ms[len(ms) // 2]
        tf = fl / (med * 1e-3) / 1e12
        by_op[name] = {"ms": round(med, 3), "tflops": round(tf, 2),
                       "frac_of_peak": round(tf / PEAK_FP64_MFMA_TFLOPS, 4), "flops": fl}
    # The dsyrk call is one kernel launch: its roofline is that launch's.
    syrk_ms = by_op["dsyrk"]["ms"]
    achieved = ops["dsyrk"][1] / (syrk_ms * 1e-3) / 1e12
    cpu = None
    if args.cpu_budget > 0:
        log("[bench] timing the CPU oracle baseline")
        v, cores, desc = blas3_cpu_baseline(hA, hT, hB, n, args.cpu_budget)
        cpu = {"value": v, "unit": "TFLOP/s", "cores": cores, "kind": "oracle", "sample": desc}
    vid = mdg.mdg_dsyrk_select_variant("L", "N", n, n)
    # HBM bytes of the dsyrk launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated), valid
    # only if taken on this kernel source.
    traffic = None
    if os.path.exists(BLAS3_TRAFFIC_FILE):
        try:
            t = json.load(open(BLAS3_TRAFFIC_FILE))
            if t.get("source_sha") == source_hash() and t.get("n") == n:
                traffic = t.get("dsyrk_bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    out = {
        "metric": "FP64 level-3 BLAS on the GEMM (dsyrk + dtrmm + dtrsm) TFLOP/s",
        "value": round(value, 3), "unit": "TFLOP/s",
        "pct_of_peak": round(100.0 * value / PEAK_FP64_MFMA_TFLOPS, 1),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded Uniform[-1,1] FP64; a well-conditioned triangle (diagonal "
                "magnitude in [1,2), off-diagonal U[-1,1)/n); resident in HBM before timing",
        "config": {"workload": f"dsyrk L N n=k={n}; dtrmm and dtrsm L L N N m=n={n}; ld = rows; "
                               "alpha = beta = 1", "flops_per_step": step_flops, "by_op": by_op},
        "roofline": {"bound": "mfma", "kernel": f"dsyrk ring kernel ({mdg.mdg_variant_name(vid)}, lower)",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4), "avg_launch_ms": syrk_ms,
                     "launches": args.steps, "traffic": traffic,
                     "algorithmic_bytes": 8.0 * (n * n + n * (n + 1))},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def synth_seed(workload):
    import synth
    return synth.seed_for(workload, 0, 0)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of CPU time for the oracle baseline (0 disables it)")
    ap.add_argument("--shapes", default="", help="comma list of sizes and/or 'skinny' (default: all)")
    ap.add_argument("--trans", default="", help="comma list of NN,NT,TN,TT (default: all four)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="force one kernel variant for every GEMM (default -1: the library's choice)")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "split", "grouped", "served", "blas3"],
                    help="sweep: the native dgemm sweep (default, the headline line); split: the "
                         "split-precision INT8 path against the native kernel; blas3: dsyrk, "
                         "dtrmm and dtrsm built on the GEMM")
    ap.add_argument("--split-size", type=int, default=8192)
    ap.add_argument("--tune", action="store_true", help="grouped: run the autotuner first")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: requests per second")
    ap.add_argument("--duration", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--budget-gb", type=int, default=64, help="served: HBM budget in GiB")
    ap.add_argument("--tune-db", default="", help="grouped: tuning database path")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes three times (the "
                         "reference kernel for scaling HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only; --gpus must be 1 (the library has no "
              "multi-GPU path: a GEMM would shard by output tiles, each GPU running this kernel)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_00076_amd as mdg
    mdg.load()
    if not torch.cuda.is_available():
        print("bench.py: no HIP device visible", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration:
        n = args.copy_calibration // 8
        src = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}), flush=True)
        return

    if args.workload == "split":
        split_workload(args, torch, mdg)
        return
    if args.workload == "grouped":
        grouped_workload(args, torch, mdg)
        return
    if args.workload == "served":
        served_workload(args, torch, mdg)
        return
    if args.workload == "blas3":
        blas3_workload(args, torch, mdg)
        return

    shapes_filter = None
    if args.shapes:
        shapes_filter = {int(s) if s.isdigit() else s for s in args.shapes.split(",")}
    probs = build_problems(torch, shapes_filter)
    if args.trans:
        keep = set(args.trans.upper().split(","))
        probs = [p for p in probs if p["transa"] + p["transb"] in keep]
    subset = bool(shapes_filter or args.trans)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        run_step(mdg, probs, variant=args.variant)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {w + 1}/{args.warmup} done")

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in probs] for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        run_step(mdg, probs, ev[s], variant=args.variant)
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    log(f"[bench] {args.steps} timed steps done in {total_ms:.1f} ms")

    step_flops = sum(flops(p) for p in probs)
    value = step_flops * args.steps / (total_ms * 1e-3) / 1e12

    # per-kernel and per-problem launch times from the per-call events
    per_kernel = {}
    per_problem = {}
    for s in range(args.steps):
        for i, p in enumerate(probs):
            ms = ev[s][i][0].elapsed_time(ev[s][i][1])
            key = kernel_key(mdg, p, args.variant)
            d = per_kernel.setdefault(key, dict(ms=0.0, flops=0.0, bytes=0.0, launches=0))
            d["ms"] += ms
            d["flops"] += flops(p)
            d["bytes"] += hbm_bytes(p)
            d["launches"] += 1
            name = f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']}"
            per_problem.setdefault(name, []).append(ms)
    dom_key = max(per_kernel, key=lambda k: per_kernel[k]["ms"])
    dom = per_kernel[dom_key]
    avg_ms = dom["ms"] / dom["launches"]
    achieved = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12

    # HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled by a
    # copy-kernel calibration), valid only if taken on this kernel source and the same launch mix.
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            t = json.load(open(TRAFFIC_FILE))
            if t.get("source_sha") == source_hash() and t.get("workload") == out_workload(probs):
                traffic = t.get("bytes_per_launch", {}).get(dom_key)
        except (OSError, ValueError):
            traffic = None

    breakdown = {}
    for name, times in per_problem.items():
        m, n, k = (int(x) for x in name.split()[1].split("x"))
        med = sorted(times)[len(times) // 2]
        breakdown[name] = round(2.0 * m * n * k / (med * 1e-3) / 1e12, 2)

    cpu = None
    if args.cpu_budget > 0:
        log("[bench] timing the CPU oracle baseline")
        v, cores, desc = cpu_baseline(probs, args.cpu_budget)
        v1, _, desc1 = cpu_baseline(probs, args.cpu_budget / 3, threads=1)
        cpu = {"value": v, "unit": "TFLOP/s", "cores": cores, "kind": "oracle", "sample": desc,
               "value_1_thread": v1, "sample_1_thread": desc1}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "pct_of_peak": round(100.0 * value / PEAK_FP64_MFMA_TFLOPS, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded Uniform[-1,1] FP64, resident in HBM before timing",
        "config": {
            "workload": "native dgemm sweep: (N|T)x(N|T) x square m=n=k in "
                        "{1024,2048,4096,4099,8192,16384} + 8192x8192x64; ld = stored rows rounded "
                        "up to a multiple of 8; alpha=beta=1" if not subset else
                        "native dgemm subset: " + ", ".join(
                            sorted({f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']}"
                                    for p in probs})),
            "gemms_per_step": len(probs),
            "flops_per_step": step_flops,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": dom_key,
            "achieved": round(achieved, 3),
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4),
            "avg_launch_ms": round(avg_ms, 4),
            "launches": dom["launches"],
            "traffic": traffic,
        },
        "cpu_baseline": cpu,
        "per_problem_tflops": breakdown,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

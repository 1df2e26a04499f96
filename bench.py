#!/usr/bin/env python3
"""FP64 GEMM benchmark on one MI355X: native dgemm sweep through the C ABI.

One step = one pass over the sweep workload: the four (transa, transb) cases of
square m = n = k in {1024, 2048, 4096, 4099, 8192, 16384} and the skinny
m = n = 8192, k = 64 (28 GEMMs), ld = stored rows rounded up to a multiple of 8,
alpha = beta = 1, Uniform[-1,1] entries drawn by the seeded generator and
resident in HBM before timing starts. value = total 2mnk flops / timed seconds.

The same line also carries, under "workloads", the other four workloads, each timed after the
sweep with its own CPU-oracle baseline: the plain NN 256^3 call (lda = ldb = ldc = 260), the
split-precision path at NN 8192^3 for exponent spreads 0, 8 and 32 against the native kernel, the
2048-GEMM grouped batch as a graph replay, and the 60-second served stream.

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


def sweep_shapes():
    """(transa, transb, m, n, k) of the sweep problems in build_problems' launch order."""
    out = [dict(transa=tr[0], transb=tr[1], m=size, n=size, k=size) for size in SQUARES for tr in TRANS]
    m, n, k = SKINNY
    return out + [dict(transa=tr[0], transb=tr[1], m=m, n=n, k=k) for tr in TRANS]


def read_counter(run_dir, counter):
    """{dispatch id: (kernel name, value)} from a rocprofv3 --pmc csv directory."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(run_dir, "*counter_collection.csv")):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, v = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, v + float(r["Counter_Value"]))
    return out


def traffic_from(dirs, copy_bytes, mdg):
    """Write TRAFFIC_FILE from four rocprofv3 --pmc runs: FETCH_SIZE and WRITE_SIZE of one sweep
    step (bench.py --steps 1 --warmup 0 --cpu-budget 0), then of the copy calibration
    (bench.py --copy-calibration copy_bytes). The sweep's GEMM dispatches are matched to its
    problems in launch order (thin-kernel launches are not GEMM dispatches here: a split
    problem's figures are its tiled block's); each counter (KiB per dispatch) is scaled by the
    factor that maps its reading for one copy of copy_bytes to the bytes the copy reads (FETCH)
    or writes (WRITE)."""
    f_dir, w_dir, cf_dir, cw_dir = dirs
    def scale(run_dir, counter):
        vals = [v for _, (name, v) in sorted(read_counter(run_dir, counter).items())]
        per = sorted(vals[-3:])[1] * 1024.0  # the median of the three copies (the last launches)
        return copy_bytes / per
    fs, ws = scale(cf_dir, "FETCH_SIZE"), scale(cw_dir, "WRITE_SIZE")
    gemm = ("dgemm_ring_kernel", "dgemm_mfma_kernel", "dgemm_wave_kernel")
    probs = sweep_shapes()
    per = {}
    for counter, sc in (("FETCH_SIZE", fs), ("WRITE_SIZE", ws)):
        rows = [v for _, (name, v) in sorted(read_counter(f_dir if counter == "FETCH_SIZE" else w_dir,
                                                             counter).items())
                if any(g in name for g in gemm)]
        if len(rows) != len(probs):
            raise SystemExit(f"{counter}: {len(rows)} GEMM dispatches for {len(probs)} problems")
        for p, v in zip(probs, rows):
            d = per.setdefault(kernel_key(mdg, p), dict(meas=0.0, alg=0.0, n=0, shapes=set()))
            d["meas"] += v * 1024.0 * sc
            if counter == "FETCH_SIZE":
                # the tiled block only, where a thin launch takes the fringe rows and columns
                _, m0, n0 = mdg.mdg_dgemm_plan(p["transa"], p["transb"], p["m"], p["n"], p["k"])
                d["alg"] += hbm_bytes(dict(p, m=m0 or p["m"], n=n0 or p["n"]))
                d["n"] += 1
                d["shapes"].add(f"{p['m']}x{p['n']}x{p['k']}")
    out = {"source_sha": source_hash(), "workload": out_workload(probs), "fetch_scale": fs,
           "write_scale": ws,
           "bytes_per_launch": {k: d["meas"] / d["n"] for k, d in sorted(per.items())},
           "algorithmic_bytes_per_launch": {k: d["alg"] / d["n"] for k, d in sorted(per.items())},
           "note": "FETCH_SIZE + WRITE_SIZE per dispatch (KiB x 1024), each times the factor that "
                   "maps the counter's reading of a device copy to the bytes it moves; averaged "
                   "over the kernel's launches in one sweep step"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(f"FETCH_SIZE x {fs:.4f}, WRITE_SIZE x {ws:.4f}")
    print("| Kernel [transposes] | launches | measured GB | algorithmic GB | ratio |")
    print("|---|---|---|---|---|")
    for k, d in sorted(per.items()):
        meas, alg = d["meas"] / d["n"], d["alg"] / d["n"]
        print(f"| `{k}` | {', '.join(sorted(d['shapes']))} | {meas / 1e9:.3f} | {alg / 1e9:.3f} | "
              f"{meas / alg:.1f} |")


def blas3_traffic_from(dirs, copy_bytes, n=8192):
    """Write BLAS3_TRAFFIC_FILE from four rocprofv3 --pmc runs as in traffic_from, the first two
    of `bench.py --workload blas3 --steps 1 --warmup 0 --cpu-budget 0`: the bytes of the dsyrk
    call's launches (the triangle-kernel launch and the n / 1024 - 1 GEMM launches before it)."""
    f_dir, w_dir, cf_dir, cw_dir = dirs
    def scale(run_dir, counter):
        vals = [v for _, (name, v) in sorted(read_counter(run_dir, counter).items())]
        return copy_bytes / (sorted(vals[-3:])[1] * 1024.0)
    fs, ws = scale(cf_dir, "FETCH_SIZE"), scale(cw_dir, "WRITE_SIZE")
    gemms = n // 1024 - 1  # GEMM launches of the call before its triangle launch
    got = {}
    for counter, d, sc in (("FETCH_SIZE", f_dir, fs), ("WRITE_SIZE", w_dir, ws)):
        rows = sorted(read_counter(d, counter).items())
        first = [i for i, (_, (name, _)) in enumerate(rows) if "dsyrk_ring_kernel" in name]
        if not first:
            raise SystemExit(f"{counter}: no dsyrk dispatch in {d}")
        i = first[0]
        call = rows[i - gemms:i + 1]
        if len(call) != gemms + 1 or not all("dgemm" in nm for _, (nm, _) in call[:-1]):
            raise SystemExit(f"{counter}: the {gemms} GEMM dispatches before the dsyrk one are missing")
        got[counter] = (sum(v for _, (_, v) in call) * 1024.0 * sc,
                        call[-1][1][1] * 1024.0 * sc, len(call))
    alg = 8.0 * (n * n + n * (n + 1))  # A read once, the triangle of C read and written
    out = {"source_sha": source_hash(), "n": n,
           "dsyrk_call_bytes": got["FETCH_SIZE"][0] + got["WRITE_SIZE"][0],
           "fetch_bytes": got["FETCH_SIZE"][0], "write_bytes": got["WRITE_SIZE"][0],
           "triangle_launch_bytes": got["FETCH_SIZE"][1] + got["WRITE_SIZE"][1],
           "launches": got["FETCH_SIZE"][2],
           "fetch_scale": fs, "write_scale": ws, "algorithmic_bytes": alg,
           "note": f"dsyrk L N n=k={n} call ({gemms} GEMM launches, then the triangle launch over "
                   "the diagonal blocks): FETCH_SIZE + WRITE_SIZE (KiB x 1024) times the factors "
                   "that map each counter's reading of a device copy to the bytes it moves"}
    with open(BLAS3_TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def out_workload(probs):
    return sorted({f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']}" for p in probs})


def flops(p):
    return 2.0 * p["m"] * p["n"] * p["k"]


def hbm_bytes(p, beta=1.0):
    """Algorithmic bytes: read op(A), op(B) once, read C if beta != 0, write C once."""
    m, n, k = p["m"], p["n"], p["k"]
    return 8.0 * (m * k + k * n + m * n * (beta != 0.0) + m * n)


def kernel_key(mdg, p, variant=-1):
    """The variant a problem launches; an automatic call whose plan splits thin fringe rows or
    columns off the tiled block (a second, thin-kernel launch) gets its own key."""
    if variant >= 0:
        return f"{mdg.mdg_variant_name(variant)}[{p['transa']}{p['transb']}]"
    v, m0, n0 = mdg.mdg_dgemm_plan(p["transa"], p["transb"], p["m"], p["n"], p["k"])
    name = mdg.mdg_variant_name(v) if v >= 0 else "thin"
    split = "+thin" if 0 <= v and (m0 < p["m"] or n0 < p["n"]) else ""
    return f"{name}{split}[{p['transa']}{p['transb']}]"


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



def host_cores():
    """(threads the oracle uses, affinity mask of this process as ranges, os.cpu_count())."""
    try:
        cpus = sorted(os.sched_getaffinity(0))
    except AttributeError:
        cpus = list(range(os.cpu_count() or 1))
    ranges, start = [], None
    for i, c in enumerate(cpus):
        if start is None:
            start = c
        if i + 1 == len(cpus) or cpus[i + 1] != c + 1:
            ranges.append(f"{start}" if start == c else f"{start}-{c}")
            start = None
    return ",".join(ranges), os.cpu_count()


def sample_lines(size: int, count: int, seed: int):
    """Sorted unique indices of rows (or columns): the edges, tile boundaries and seeded ones."""
    import numpy as np

    import synth
    fixed = [0, 1, 15, 16, 63, 64, 127, 128, 129, 255, 256, size // 2, size - 2, size - 1]
    rnd = synth.rng(seed).integers(0, size, count).tolist() if size > 0 else []
    return np.array(sorted({i for i in fixed + rnd if 0 <= i < size}), dtype=np.int64)


def oracle_lines(hA, hB, hC, m, n, k, lda, ldb, ldc, alpha, beta, R, S, fn="dgemm", at=None):
    """The oracle's full rows R and full columns S of C for an NN problem on host storage, and the
    error denominators D of the same entries. The needed rows of A and columns of B are copied out
    (data movement only; `at` may hold A transposed to k-contiguous rows already), so the oracle
    evaluates exactly the products and order of the whole problem, each entry a dot product over
    contiguous memory. Returns (rows |R| x n, D rows, cols m x |S|, D cols, multiply-adds)."""
    import numpy as np

    import oracle
    import synth
    Av = synth.view2d(hA, m, k, lda)
    Bv = synth.view2d(hB, k, n, ldb)
    C0 = synth.view2d(hC, m, n, ldc)
    f = getattr(oracle, fn)
    ar = np.ascontiguousarray(Av[R, :]).reshape(-1)          # op(A)[R, :]^T stored k x |R|
    c0r = np.asfortranarray(C0[R, :]).reshape(-1, order="F")
    cr = c0r.copy()
    assert f("T", "N", len(R), n, k, alpha, ar, k, hB, ldb, beta, cr, len(R)) == 0
    dr = np.zeros(len(R) * n)
    assert oracle.absden("T", "N", len(R), n, k, alpha, ar, k, hB, ldb, beta, c0r, len(R), dr,
                         len(R)) == 0
    bs = np.asfortranarray(Bv[:, S]).reshape(-1, order="F")  # op(B)[:, S] stored k x |S|
    c0s = np.asfortranarray(C0[:, S]).reshape(-1, order="F")
    if at is None:
        at = np.ascontiguousarray(Av).reshape(-1)            # op(A)^T stored k x m
    cs = c0s.copy()
    assert f("T", "N", m, len(S), k, alpha, at, k, bs, k, beta, cs, m) == 0
    ds = np.zeros(m * len(S))
    assert oracle.absden("T", "N", m, len(S), k, alpha, at, k, bs, k, beta, c0s, m, ds, m) == 0
    macs = float(len(R) * n + m * len(S)) * k
    return (cr.reshape(n, len(R)).T, dr.reshape(n, len(R)).T, cs.reshape(len(S), m).T,
            ds.reshape(len(S), m).T, macs)


def max_rel_err(got, ref, D):
    """max |got - ref| / D (entries with D = 0 must be equal, else inf)."""
    import numpy as np
    diff = np.abs(got - ref)
    zero = D == 0
    if np.any(zero & (diff != 0)) or np.any(np.isnan(diff)):
        return float("inf")
    return float(np.max(np.where(zero, 0.0, diff / np.where(zero, 1.0, D)))) if diff.size else 0.0

# (phi, nslices, nmoduli) that reach err <= 1e-13 at 8192^3: slice counts for the slice scheme,
# modulus counts for the Chinese-remainder scheme
SPLIT_CASES = [(0, 7, 14), (8, 8, 15), (32, 10, 16)]
INT8_PEAK_TOPS = 5000.0


def events_ms(torch, fn, reps, warmup):
    """Average milliseconds per call of fn() over `reps` calls on the current stream (HIP events
    around the whole run), after `warmup` untimed calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def split_result(args, torch, mdg):
    """Workload 3: split-precision dgemm on the INT8 matrix cores against the native FP64 kernel,
    NN 8192^3, phi in {0, 8, 32}, by both schemes: slices (Ozaki scheme I, S(S+1)/2 slice products)
    and the Chinese remainder theorem (scheme II, one product per modulus). Times each whole call,
    its operand-splitting steps alone, and the native call; in the CPU-baseline leg the oracle
    computes sampled full rows and columns, which are timed and also give every result's error
    (and a doubled-precision sample gives the true error)."""
    import numpy as np

    import synth
    m = n = k = args.split_size
    cases, cpu_parts = [], []
    cpu_flops = cpu_s = 0.0
    fl = 2.0 * m * n * k
    for phi, S, N in SPLIT_CASES:
        dist = "scaled" if phi else "uniform"
        p = synth.problem(3, phi, "N", "N", m, n, k, ld_rule=synth.ld_round8, dist=dist, phi=phi)
        lda, ldb, ldc = p["lda"], p["ldb"], p["ldc"]
        dA, dB, dC0 = (torch.from_numpy(p[x]).cuda() for x in "ABC")
        dC = dC0.clone()
        ws_s = mdg.mdg_dgemm_split_workspace_size(m, n, k, S)
        ws_c = mdg.mdg_dgemm_crt_workspace_size(m, n, k, N)
        ws = torch.empty(max(ws_s, ws_c), dtype=torch.uint8, device="cuda")
        rp, kp = (m + 127) // 128 * 128, (k + 63) // 64 * 64
        sl = torch.empty(max(S, N) * rp * kp, dtype=torch.int8, device="cuda")
        ex = torch.empty(max(m, n), dtype=torch.int32, device="cuda")
        bits = mdg.mdg_crt_bits(k, N)

        def check(st):
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))

        def slices_call():
            check(mdg.mdg_dgemm_split("N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 1.0, dC, ldc, S, ws,
                                      ws_s))

        def crt_call():
            check(mdg.mdg_dgemm_crt("N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 1.0, dC, ldc, N, ws,
                                    ws_c))

        def native_call():
            check(mdg.mdg_dgemm("N", "N", m, n, k, 1.0, dA, lda, dB, ldb, 1.0, dC, ldc))

        def slicing_only():
            check(mdg.mdg_split_slices(0, "N", m, k, dA, lda, S, sl, ex))
            check(mdg.mdg_split_slices(1, "N", n, k, dB, ldb, S, sl, ex))

        def residues_only():
            check(mdg.mdg_crt_residues(0, "N", m, k, dA, lda, N, bits, sl, ex))
            check(mdg.mdg_crt_residues(1, "N", n, k, dB, ldb, N, bits, sl, ex))

        t = {name: events_ms(torch, fn, args.steps, args.warmup)
             for name, fn in (("slices", slices_call), ("crt", crt_call), ("native", native_call),
                              ("slicing", slicing_only), ("residues", residues_only))}
        # one result of each path from the original C, for the error figures
        outs = {}
        for name, fn in (("slices", slices_call), ("crt", crt_call), ("native", native_call)):
            dC.copy_(dC0)
            fn()
            outs[name] = dC.view(n, ldc)[:, :m].T.cpu().numpy()
        del dA, dB, dC, dC0, ws, sl, ex
        torch.cuda.empty_cache()
        sp = S * (S + 1) // 2
        case = {
            "phi": phi, "native_ms": round(t["native"], 3),
            "native_tflops": round(fl / (t["native"] * 1e-3) / 1e12, 2),
            "crt": {"nmoduli": N, "bits": bits, "int8_products": N, "ms": round(t["crt"], 3),
                    "residues_ms": round(t["residues"], 3),
                    "products_and_recombination_ms": round(t["crt"] - t["residues"], 3),
                    "tflops_equiv": round(fl / (t["crt"] * 1e-3) / 1e12, 2),
                    "speedup_vs_native": round(t["native"] / t["crt"], 3),
                    "int8_tops_excl_residues": round(N * fl / ((t["crt"] - t["residues"]) * 1e-3)
                                                     / 1e12, 1),
                    "max_err_vs_oracle": None, "true_err_vs_doubled_precision": None},
            "slices": {"nslices": S, "int8_products": sp, "ms": round(t["slices"], 3),
                       "slicing_ms": round(t["slicing"], 3),
                       "gemm_kernel_ms": round(t["slices"] - t["slicing"], 3),
                       "tflops_equiv": round(fl / (t["slices"] * 1e-3) / 1e12, 2),
                       "speedup_vs_native": round(t["native"] / t["slices"], 3),
                       "int8_tops_gemm_kernel": round(sp * fl / ((t["slices"] - t["slicing"]) * 1e-3)
                                                      / 1e12, 1),
                       "max_err_vs_oracle": None, "true_err_vs_doubled_precision": None},
            "native_max_err_vs_oracle": None,
        }
        if args.cpu_budget > 0:
            # CPU-baseline leg: the oracle on sampled full rows and columns (timed), whose values
            # also state every GPU result's error.
            R = sample_lines(m, 4, synth.seed_for(3, phi, 5))
            Sx = sample_lines(n, 4, synth.seed_for(3, phi, 6))
            at = np.ascontiguousarray(synth.view2d(p["A"], m, k, lda)).reshape(-1)
            t0 = time.perf_counter()
            ref_r, d_r, ref_c, d_c, macs = oracle_lines(p["A"], p["B"], p["C"], m, n, k, lda, ldb,
                                                        ldc, 1.0, 1.0, R, Sx, at=at)
            dt = time.perf_counter() - t0
            cpu_flops += 2.0 * macs  # the denominators' pass is not counted
            cpu_s += dt
            cpu_parts.append(f"phi={phi}: {len(R)} rows + {len(Sx)} columns ({dt:.1f} s)")

            def err(c):
                return float(f"{max(max_rel_err(c[R, :], ref_r, d_r), max_rel_err(c[:, Sx], ref_c, d_c)):.3g}")
            case["crt"]["max_err_vs_oracle"] = err(outs["crt"])
            case["slices"]["max_err_vs_oracle"] = err(outs["slices"])
            case["native_max_err_vs_oracle"] = err(outs["native"])
            R2, S2 = R[:3], Sx[-3:]
            dd_r, _, dd_c, _, _ = oracle_lines(p["A"], p["B"], p["C"], m, n, k, lda, ldb, ldc, 1.0,
                                               1.0, R2, S2, fn="dgemm_dd", at=at)
            d_r2, d_c2 = d_r[:3], d_c[:, -3:]
            for name in ("crt", "slices"):
                c = outs[name]
                case[name]["true_err_vs_doubled_precision"] = float(
                    f"{max(max_rel_err(c[R2, :], dd_r, d_r2), max_rel_err(c[:, S2], dd_c, d_c2)):.3g}")
            del at
        cases.append(case)
        log(f"[bench] split phi={phi}: {case}")
        del outs, p
    cpu = None
    if cpu_s > 0:
        mask, ncpu = host_cores()
        import oracle
        cpu = {"value": cpu_flops / cpu_s / 1e12, "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "affinity": mask, "cpu_count": ncpu, "kind": "oracle",
               "sample": "oracle on sampled full rows and columns of C of each 8192^3 case: " +
                         "; ".join(cpu_parts)}
    best = max(cases, key=lambda c: c["crt"]["tflops_equiv"])
    return {
        "workload": f"split-precision dgemm NN {m}x{n}x{k}, ld rounded to 8, alpha=beta=1, "
                    "entries u*2^e, u ~ U[-1,1), e ~ U{-phi..phi}; Chinese-remainder scheme "
                    "(14/15/16 moduli) and slice scheme (7/8/10 slices) against native FP64",
        "unit": "TFLOP/s (FP64-equivalent)",
        "cases": cases,
        "roofline": {"bound": "mfma", "kernel": f"CRT modular products and recombination, "
                                                f"{best['crt']['nmoduli']} moduli (phi={best['phi']})",
                     "achieved": best["crt"]["int8_tops_excl_residues"], "peak": INT8_PEAK_TOPS,
                     "unit": "TOP/s (int8)",
                     "frac": round(best["crt"]["int8_tops_excl_residues"] / INT8_PEAK_TOPS, 4),
                     "note": "time = whole CRT call minus the two residue steps timed alone (the "
                             "recombination kernel included)"},
        "cpu_baseline": cpu,
    }


def split_workload(args, torch, mdg):
    r = split_result(args, torch, mdg)
    best = max(r["cases"], key=lambda c: c["crt"]["tflops_equiv"])
    out = {
        "metric": METRIC + " (split-precision leg)",
        "value": best["crt"]["tflops_equiv"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8 slices, f64 recombination",
        "data": "synthetic: seeded u*2^e, u ~ U[-1,1), e ~ U{-phi..phi}",
        "config": {"workload": r["workload"], "cases": r["cases"]},
        "roofline": r["roofline"], "cpu_baseline": r["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


def grouped_problems(count=2048, lo=16, hi=512, seed_variant=0):
    """Workload of 2048 independent GEMMs: m, n, k log-uniform integers in [lo, hi], transposes
    iid, alpha and beta ~ U[-1, 1), tight leading dimensions, entries U[-1, 1)."""
    import synth
    return synth.grouped_batch(count, lo, hi, seed_variant)


def grouped_result(args, torch, mdg):
    """Workload 4: 2048 uneven GEMMs as one grouped launch replayed from a graph, against the
    eager grouped launch and against one mdg_dgemm launch per GEMM."""
    import oracle
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

    plan = GroupedPlan(gemms, tuner.classes_for(gemms, policy), policy["schedule"])
    eager_grouped = events_ms(torch, lambda: plan.launch(policy["grid"]), args.steps, args.warmup)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.launch(policy["grid"])
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch(policy["grid"])
    graph_ms = events_ms(torch, graph.replay, args.steps, args.warmup)

    def per_gemm():
        for g in gemms:
            st = mdg.mdg_dgemm(g["transa"], g["transb"], g["m"], g["n"], g["k"], g["alpha"],
                               g["A"], g["lda"], g["B"], g["ldb"], g["beta"], g["C"], g["ldc"])
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))
    separate_ms = events_ms(torch, per_gemm, max(1, args.steps // 4), 1)
    value = total_flops / (graph_ms * 1e-3) / 1e12
    cpu = None
    if args.cpu_budget > 0:
        # the oracle on the batch's GEMMs in order until a share of the budget is spent
        import numpy as np
        t_spent, fl, count = 0.0, 0.0, 0
        for p in probs:
            c = p["C"].copy()
            t0 = time.perf_counter()
            assert oracle.dgemm(p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"],
                                p["A"], p["lda"], p["B"], p["ldb"], p["beta"], c, p["ldc"]) == 0
            t_spent += time.perf_counter() - t0
            fl += 2.0 * p["m"] * p["n"] * p["k"]
            count += 1
            if t_spent > args.cpu_budget / 4:
                break
        del np
        mask, ncpu = host_cores()
        cpu = {"value": fl / t_spent / 1e12, "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "affinity": mask, "cpu_count": ncpu, "kind": "oracle",
               "sample": f"oracle on the first {count} GEMMs of the batch ({t_spent:.1f} s)"}
    return {
        "workload": "2048 independent dgemm, m,n,k log-uniform integers in [16,512], transposes "
                    "iid, alpha,beta ~ U[-1,1), tight ld; one grouped persistent launch replayed "
                    "from a graph",
        "policy": policy, "tiles": plan.num_tiles,
        "total_flops": total_flops, "algorithmic_bytes": total_bytes,
        "graph_replay_ms": round(graph_ms, 4),
        "tflops": round(value, 3),
        "eager_grouped_ms": round(eager_grouped, 4),
        "separate_launches_ms": round(separate_ms, 4),
        "speedup_vs_separate": round(separate_ms / graph_ms, 2),
        "roofline": {"bound": "hbm", "achieved": round(total_bytes / (graph_ms * 1e-3) / 1e9, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(total_bytes / (graph_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "mfma_frac": round(value / PEAK_FP64_MFMA_TFLOPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }


def grouped_workload(args, torch, mdg):
    r = grouped_result(args, torch, mdg)
    out = {
        "metric": METRIC + " (grouped-launch leg)",
        "value": r["tflops"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["graph_replay_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded U[-1,1) FP64, shapes log-uniform in [16,512]",
        "config": {k: r[k] for k in ("workload", "policy", "tiles", "total_flops",
                                     "algorithmic_bytes")},
        **{k: r[k] for k in ("graph_replay_ms", "eager_grouped_ms", "separate_launches_ms",
                             "speedup_vs_separate", "roofline", "cpu_baseline")},
    }
    print(json.dumps(out), flush=True)


def served_result(args, torch, mdg):
    """Workload 5: a Poisson stream of dgemm requests through the continuous-batching server."""
    import numpy as np

    import oracle
    import synth
    from paper_1609_00076_amd import serve
    reqs = serve.make_stream(args.rate, args.duration, seed=synth_seed(5), lo=32, hi=4096,
                             split_fraction=0.2, phi=8)
    log(f"[bench] serving {len(reqs)} requests over {args.duration} s")
    warm = serve.make_stream(200, 0.5, seed=synth_seed(5) + 1, lo=32, hi=512)
    srv = serve.Server(budget_bytes=args.budget_gb << 30)
    srv.run(warm)  # warm-up of allocator and streams
    stats = srv.run(reqs)
    s = stats.summary()
    log(f"[bench] served: {s}")
    cpu = None
    if args.cpu_budget > 0:
        # the oracle on the stream's first requests (same shapes, seeded host data), in order,
        # until a share of the budget is spent
        t_spent, fl, count = 0.0, 0.0, 0
        for r in reqs:
            ra, ca = r.stored("A")
            rb, cb = r.stored("B")
            g = synth.rng(r.seed % (1 << 32))
            A, B, C = (g.uniform(-1, 1, max(1, x * y)) for x, y in ((ra, ca), (rb, cb), (r.m, r.n)))
            t0 = time.perf_counter()
            assert oracle.dgemm(r.transa, r.transb, r.m, r.n, r.k, r.alpha, A, max(1, ra), B,
                                max(1, rb), r.beta, C, max(1, r.m)) == 0
            t_spent += time.perf_counter() - t0
            fl += r.flops
            count += 1
            if t_spent > args.cpu_budget / 4:
                break
        del np
        mask, ncpu = host_cores()
        cpu = {"value": fl / t_spent / 1e12, "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "affinity": mask, "cpu_count": ncpu, "kind": "oracle",
               "sample": f"oracle on the first {count} requests of the stream ({t_spent:.1f} s)"}
    return {
        "workload": f"Poisson {args.rate:g} req/s for {args.duration:g} s, m,n,k log-uniform in "
                    "[32,4096], transposes iid, 80% native, 20% split (phi=8, Chinese-remainder "
                    f"scheme with {serve.SPLIT_MODULI[8]} moduli), HBM budget {args.budget_gb} GiB",
        "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"], "aggregate_tflops": s["aggregate_tflops"],
        "served": s, "cpu_baseline": cpu,
    }


def served_workload(args, torch, mdg):
    r = served_result(args, torch, mdg)
    s = r["served"]
    out = {
        "metric": METRIC + " (served-stream leg)",
        "value": s["aggregate_tflops"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * s["wall_s"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: operands filled on the device from per-request seeds",
        "config": {"workload": r["workload"]},
        "served": s, "cpu_baseline": r["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


PLAIN = dict(m=256, n=256, k=256, ld=260, alpha=1.5, beta=0.5)


def plain_result(args, torch, mdg):
    """Workload 1: NN 256^3 with lda = ldb = ldc = 260, alpha = 1.5, beta = 0.5, uniform entries
    (and the integer-valued variant for a bit-exact check in the CPU-baseline leg)."""
    import numpy as np

    import synth
    m, n, k, ld, alpha, beta = (PLAIN[x] for x in ("m", "n", "k", "ld", "alpha", "beta"))
    out = {"workload": f"dgemm NN {m}x{n}x{k}, lda=ldb=ldc={ld}, alpha={alpha}, beta={beta}, "
                       "U[-1,1) entries"}
    results = {}
    for dist in ("uniform", "int"):
        p = synth.problem(1, 0, "N", "N", m, n, k, ld_rule=lambda r: ld, dist=dist)
        dA, dB, dC0 = (torch.from_numpy(p[x]).cuda() for x in "ABC")
        dC = dC0.clone()

        def call():
            st = mdg.mdg_dgemm("N", "N", m, n, k, alpha, dA, ld, dB, ld, beta, dC, ld)
            if st:
                raise RuntimeError(mdg.mdg_status_string(st))
        if dist == "uniform":
            reps = max(200, 20 * args.steps)
            # per-call events: the median call, and the back-to-back average
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for _ in range(args.warmup + 5):
                call()
            torch.cuda.synchronize()
            for e0, e1 in ev:
                e0.record()
                call()
                e1.record()
            torch.cuda.synchronize()
            t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
            med_us = 1e3 * t[len(t) // 2]
            avg_us = 1e3 * events_ms(torch, call, reps, 0)
            fl = 2.0 * m * n * k
            by = 8.0 * (2 * m * k + 2 * m * n)
            out.update({
                "median_us": round(med_us, 2), "back_to_back_avg_us": round(avg_us, 2),
                "tflops": round(fl / (med_us * 1e-6) / 1e12, 3),
                "frac_of_fp64_mfma_peak": round(fl / (med_us * 1e-6) / 1e12 / PEAK_FP64_MFMA_TFLOPS, 5),
                "gbs": round(by / (med_us * 1e-6) / 1e9, 1),
                "frac_of_hbm_peak": round(by / (med_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 5),
                "variant": mdg.mdg_variant_name(mdg.mdg_select_variant("N", "N", m, n, k, alpha,
                                                                      beta)),
            })
        dC.copy_(dC0)
        call()
        results[dist] = (p, synth.view2d(dC.cpu().numpy(), m, n, ld).copy())
    cpu = None
    if args.cpu_budget > 0:
        # CPU-baseline leg: the oracle on the same problem, repeated; its values also check the
        # GPU results (bit-exact on integers, error relative to D on uniform entries)
        import oracle
        p, got = results["uniform"]
        reps, t_spent = 0, 0.0
        while t_spent < min(2.0, args.cpu_budget / 8):
            ref = p["C"].copy()
            t0 = time.perf_counter()
            assert oracle.dgemm("N", "N", m, n, k, alpha, p["A"], ld, p["B"], ld, beta, ref, ld) == 0
            t_spent += time.perf_counter() - t0
            reps += 1
        D = np.zeros(m * n)
        assert oracle.absden("N", "N", m, n, k, alpha, p["A"], ld, p["B"], ld, beta, p["C"], ld, D,
                             m) == 0
        out["max_err_vs_oracle"] = float(f"{max_rel_err(got, synth.view2d(ref, m, n, ld), D.reshape(n, m).T):.3g}")
        pi, goti = results["int"]
        refi = pi["C"].copy()
        assert oracle.dgemm("N", "N", m, n, k, alpha, pi["A"], ld, pi["B"], ld, beta, refi, ld) == 0
        out["integer_variant_bit_exact"] = bool(np.array_equal(goti, synth.view2d(refi, m, n, ld)))
        mask, ncpu = host_cores()
        cpu = {"value": reps * 2.0 * m * n * k / t_spent / 1e12, "unit": "TFLOP/s",
               "cores": oracle.get_threads(), "affinity": mask, "cpu_count": ncpu,
               "kind": "oracle", "sample": f"oracle on the whole problem, {reps} times "
                                           f"({t_spent:.1f} s)"}
    out["cpu_baseline"] = cpu
    return out


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
    # The roofline is the dsyrk call's: at n = 8192 the GEMMs between its diagonal blocks (seven
    # launches) and one launch of the triangle kernel over the eight diagonal blocks.
    syrk_ms = by_op["dsyrk"]["ms"]
    achieved = ops["dsyrk"][1] / (syrk_ms * 1e-3) / 1e12
    cpu = None
    if args.cpu_budget > 0:
        log("[bench] timing the CPU oracle baseline")
        v, cores, desc = blas3_cpu_baseline(hA, hT, hB, n, args.cpu_budget)
        cpu = {"value": v, "unit": "TFLOP/s", "cores": cores, "kind": "oracle", "sample": desc}
    vid = mdg.mdg_dsyrk_select_variant("L", "N", n, n)
    # HBM bytes of the dsyrk call's launches (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated),
    # valid only if taken on this kernel source.
    traffic = None
    if os.path.exists(BLAS3_TRAFFIC_FILE):
        try:
            t = json.load(open(BLAS3_TRAFFIC_FILE))
            if t.get("source_sha") == source_hash() and t.get("n") == n:
                traffic = t.get("dsyrk_call_bytes")
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
        "roofline": {"bound": "mfma",
                     "kernel": f"dsyrk call: {n // 1024 - 1} GEMM launches between the diagonal "
                               f"blocks, then the triangle kernel ({mdg.mdg_variant_name(vid)}, "
                               f"lower) over {n // 1024} diagonal blocks of order 1024",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4), "avg_call_ms": syrk_ms,
                     "calls": args.steps, "traffic": traffic,
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
    ap.add_argument("--workload", default="all",
                    choices=["all", "sweep", "plain", "split", "grouped", "served", "blas3"],
                    help="all (default): the native dgemm sweep (the headline value) and, in the "
                         "same line, the plain 256^3 call, the split-precision path, the grouped "
                         "batch and the served stream; sweep: the sweep alone; split, grouped, "
                         "served: one of those alone; blas3: dsyrk, dtrmm and dtrsm on the GEMM")
    ap.add_argument("--split-size", type=int, default=8192)
    ap.add_argument("--tune", action="store_true", help="grouped: run the autotuner first")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: requests per second")
    ap.add_argument("--duration", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--budget-gb", type=int, default=64, help="served: HBM budget in GiB")
    ap.add_argument("--tune-db", default="", help="grouped: tuning database path")
    ap.add_argument("--traffic-from", default="", metavar="F,W,CF,CW",
                    help="write profiles/hbm_traffic.json from four rocprofv3 --pmc output "
                         "directories (sweep FETCH_SIZE, sweep WRITE_SIZE, copy FETCH_SIZE, copy "
                         "WRITE_SIZE; the copy of --copy-calibration bytes); no GPU needed")
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
    if args.traffic_from:
        if args.workload == "blas3":
            blas3_traffic_from(args.traffic_from.split(","), args.copy_calibration or (1 << 30))
        else:
            traffic_from(args.traffic_from.split(","), args.copy_calibration or (1 << 30), mdg)
        return
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

    if args.workload == "plain":
        print(json.dumps(plain_result(args, torch, mdg)), flush=True)
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

    # The skinny GEMM against the reachable streaming rate: the library's own C := beta*C kernel
    # (alpha = 0 takes it; a grid-stride read and write of C) on the same C, timed the same way.
    skinny = None
    sk = [p for p in probs if p["k"] == SKINNY[2]]
    if sk:
        p0 = sk[0]
        m, n = p0["m"], p0["n"]
        def st():
            if mdg.mdg_dgemm("N", "N", m, n, p0["k"], 0.0, None, m, None, p0["k"], 0.5, p0["C"],
                             p0["ldc"]):
                raise RuntimeError("C := beta*C refused")
        stream_ms = events_ms(torch, st, 20, 3)
        stream_tbs = 2.0 * 8.0 * m * n / (stream_ms * 1e-3) / 1e12
        gemm_tbs = {}
        for p in sk:
            name = f"{p['transa']}{p['transb']} {p['m']}x{p['n']}x{p['k']}"
            med = sorted(per_problem[name])[len(per_problem[name]) // 2]
            gemm_tbs[p["transa"] + p["transb"]] = round(hbm_bytes(p) / (med * 1e-3) / 1e12, 3)
        skinny = {"shape": f"{m}x{n}x{p0['k']}",
                  "stream_kernel": "C := beta*C (the library's alpha = 0 path), same C",
                  "stream_TBps": round(stream_tbs, 3), "gemm_TBps": gemm_tbs,
                  "frac_of_stream": {t: round(v / stream_tbs, 3) for t, v in gemm_tbs.items()},
                  "frac_of_hbm_peak": {t: round(v / (PEAK_HBM_GBS / 1e3), 3)
                                       for t, v in gemm_tbs.items()}}

    cpu = None
    if args.cpu_budget > 0:
        log("[bench] timing the CPU oracle baseline")
        v, cores, desc = cpu_baseline(probs, args.cpu_budget)
        v1, _, desc1 = cpu_baseline(probs, args.cpu_budget / 3, threads=1)
        mask, ncpu = host_cores()
        cpu = {"value": v, "unit": "TFLOP/s", "cores": cores, "affinity": mask, "cpu_count": ncpu,
               "kind": "oracle", "sample": desc, "value_1_thread": v1,
               "sample_1_thread": desc1}
    workload_desc = ("native dgemm sweep: (N|T)x(N|T) x square m=n=k in "
                     "{1024,2048,4096,4099,8192,16384} + 8192x8192x64; ld = stored rows rounded "
                     "up to a multiple of 8; alpha=beta=1" if not subset else
                     "native dgemm subset: " + ", ".join(out_workload(probs)))
    n_gemms = len(probs)
    del probs, ev
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    workloads = None
    if args.workload == "all" and not subset:
        workloads = {}
        for name, fn in (("plain_256", plain_result), ("split_8192", split_result),
                         ("grouped_2048", grouped_result), ("served", served_result)):
            log(f"[bench] workload {name}")
            workloads[name] = fn(args, torch, mdg)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()

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
            "workload": workload_desc,
            "gemms_per_step": n_gemms,
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
        "skinny_vs_stream": skinny,
    }
    if workloads is not None:
        out["workloads"] = workloads
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Autotuner for grouped dgemm launches: measured search over tile classes, schedules and grids.

A policy is (tile, threshold, schedule, grid). With workgroup tiles ("block"), GEMM i uses the
32x32 tile (class 1) when min(m_i, n_i) < threshold and the 64x64 tile (class 0) otherwise; with
wave tiles ("wave") every GEMM uses class 2. The tile list is in natural or largest-first (LPT)
order; `grid` persistent workgroups walk it. Each candidate is timed as a
captured graph of one grouped launch, replayed; the fastest is kept. Results are stored in a JSON
database keyed by device architecture, HIP version and a workload signature, and read back by
`best_policy`.
"""
from __future__ import annotations

import json
import os

from . import binding as b
from .grouped import GroupedPlan

DB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_db.json")
THRESHOLDS = (0, 40, 64, 96, 160, 1 << 30)
SCHEDULES = (b.MDG_SCHEDULE_NATURAL, b.MDG_SCHEDULE_LPT)
GRIDS = (256, 512, 1024, 2048)
FINALISTS = 4  # candidates timed a second time, with three times the replays
DEFAULT_POLICY = {"tile": "block", "threshold": 48, "schedule": b.MDG_SCHEDULE_LPT, "grid": 1024}
# Signature of the batched workload: 2048 GEMMs, m, n, k log-uniform in [16, 512].
GROUPED_SIGNATURE = "grouped|2048|mnk~logU[16,512]|trans iid|tight ld"


def classes_for(gemms, policy):
    """Tile class of each GEMM under `policy` (a policy dict, or a bare threshold): with
    tile "wave" every GEMM takes the 32x32 wave tile (class 2); otherwise class 1 (32x32
    workgroup tile) below the min(m, n) threshold and class 0 (64x64) from it on."""
    if isinstance(policy, dict) and policy.get("tile") == "wave":
        return [2] * len(gemms)
    threshold = policy["threshold"] if isinstance(policy, dict) else policy
    return [1 if min(g["m"], g["n"]) < threshold else 0 for g in gemms]


def device_key(signature: str) -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    return f"{arch}|hip{torch.version.hip}|{signature}"


def time_policy(gemms, policy, reps=10, warmup=3):
    """Milliseconds per replay of a graph holding one grouped launch under `policy`."""
    import torch
    plan = GroupedPlan(gemms, classes_for(gemms, policy), policy["schedule"])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warmup):
            plan.launch(policy["grid"])
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch(policy["grid"])
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def candidates(thresholds=THRESHOLDS, schedules=SCHEDULES, grids=GRIDS, wave=True):
    """Policies the tuner times: workgroup tiles for every threshold, schedule and grid, and (with
    `wave`) the wave tiles for every schedule and grid."""
    pols = [{"tile": "block", "threshold": th, "schedule": sc, "grid": gr}
            for th in thresholds for sc in schedules for gr in grids]
    if wave:
        pols += [{"tile": "wave", "threshold": 0, "schedule": sc, "grid": gr}
                 for sc in schedules for gr in grids]
    return pols


def tune_grouped(gemms, signature, thresholds=THRESHOLDS, schedules=SCHEDULES, grids=GRIDS,
                 reps=10, db_path=DB_PATH, log=None, policies=None):
    """Time every candidate policy on `gemms` (or the given `policies`), store the best under
    `signature`, return it."""
    results = []
    for pol in policies or candidates(thresholds, schedules, grids):
        ms = time_policy(gemms, pol, reps=reps)
        results.append({**pol, "ms": round(ms, 5)})
        if log:
            log(f"[tune] {pol} {ms:.4f} ms")
    # The leaders are often within a few per cent of each other: time the best few again, longer,
    # and choose among those second timings.
    keys = ("tile", "threshold", "schedule", "grid")
    for r in sorted(results, key=lambda r: r["ms"])[:FINALISTS]:
        pol = {k: r[k] for k in keys}
        r["ms_final"] = round(time_policy(gemms, pol, reps=3 * reps), 5)
        if log:
            log(f"[tune] finalist {pol} {r['ms_final']:.4f} ms")
    best = min((r for r in results if "ms_final" in r), key=lambda r: r["ms_final"])
    entry = {"policy": {k: best[k] for k in keys}, "ms": best["ms_final"], "candidates": results}
    db = load_db(db_path)
    db[device_key(signature)] = entry
    with open(db_path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    return entry


def load_db(db_path=DB_PATH):
    if os.path.exists(db_path):
        with open(db_path) as f:
            return json.load(f)
    return {}


def best_policy(signature, db_path=DB_PATH):
    """The stored policy for this device and signature, else the default one."""
    entry = load_db(db_path).get(device_key(signature))
    return dict(entry["policy"]) if entry else dict(DEFAULT_POLICY)

"""GPU parity of grouped (persistent, batched) dgemm launches, eager and graph-replayed.

Every GEMM of a batch is checked against the CPU oracle (1e-13 relative to D; bit-exact on
integer-valued inputs) and against the same GEMM run alone through mdg_dgemm_ex with the variant
whose tile its class uses (bitwise: same tile code, same k order). Graph replays are checked one
by one, with unrelated eager work and a reset of C between them.
"""
import numpy as np
import pytest

import synth
from gpu_util import TOL, logical, rel_err, run_oracle, same_bits

pytestmark = pytest.mark.gpu


def _batch(seed, count, lo, hi, dist="uniform", special=False):
    """Seeded GEMMs with log-uniform sizes, random transposes, tight leading dimensions."""
    g = synth.rng(synth.seed_for(40, seed, 9))
    m = synth.log_uniform_int(g, lo, hi, count)
    n = synth.log_uniform_int(g, lo, hi, count)
    k = synth.log_uniform_int(g, lo, hi, count)
    ta = g.integers(0, 2, count)
    tb = g.integers(0, 2, count)
    ab = g.uniform(-1, 1, (count, 2))
    probs = []
    for i in range(count):
        p = synth.problem(40, seed * 10000 + i, "NT"[ta[i]], "NT"[tb[i]], int(m[i]), int(n[i]),
                          int(k[i]), ld_rule=synth.ld_tight, dist=dist)
        alpha, beta = float(ab[i, 0]), float(ab[i, 1])
        if dist == "int":
            alpha, beta = float(np.round(alpha * 4) / 2), float(np.round(beta * 4) / 2)
        p["alpha"], p["beta"] = alpha, beta
        probs.append(p)
    if special:
        probs[0]["alpha"] = 0.0             # scale only
        probs[1]["alpha"], probs[1]["beta"] = 0.0, 1.0  # quick return: untouched
        probs[2]["k"] = 0                   # k = 0: C := beta*C
        probs[2]["lda"] = max(1, probs[2]["m"]) if probs[2]["transa"] == "N" else 1
        probs[2]["ldb"] = 1 if probs[2]["transb"] == "N" else max(1, probs[2]["n"])
        probs[3]["beta"] = 0.0              # old C never read
        logical(probs[3]["C"], probs[3]["m"], probs[3]["n"], probs[3]["ldc"])[:, :] = np.nan
    return probs


def _to_device(probs):
    import torch
    gemms = []
    for p in probs:
        gemms.append(dict(transa=p["transa"], transb=p["transb"], m=p["m"], n=p["n"], k=p["k"],
                          alpha=p["alpha"], beta=p["beta"], lda=p["lda"], ldb=p["ldb"],
                          ldc=p["ldc"], A=torch.from_numpy(p["A"]).cuda(),
                          B=torch.from_numpy(p["B"]).cuda(), C=torch.from_numpy(p["C"]).cuda()))
    return gemms


def _check_against_oracle(probs, gemms, exact):
    for i, (p, g) in enumerate(zip(probs, gemms)):
        got = g["C"].cpu().numpy()
        ref, D = run_oracle(p, p["alpha"], p["beta"])
        m, n, ldc = p["m"], p["n"], p["ldc"]
        gl, rl = logical(got, m, n, ldc), logical(ref, m, n, ldc)
        tag = f"GEMM {i}: {p['transa']}{p['transb']} {m}x{n}x{p['k']}"
        if exact:
            assert same_bits(gl, rl), tag
        else:
            assert rel_err(gl.T, rl.T, D) <= TOL, tag
        if ldc > m:
            assert np.all(got.view(np.uint64).reshape(n, ldc)[:, m:] == synth.PAD_C_BITS), tag


def _variant_of_class(cls):
    import paper_1609_00076_amd as mdg
    names = {0: "mfma_f64_64x64x16_w32x32", 1: "mfma_f64_32x32x16_w16x16",
             2: "wave_f64_64x64x8_w32x32"}
    for v in range(mdg.mdg_num_variants()):
        if mdg.mdg_variant_name(v) == names[cls]:
            return v
    raise AssertionError("variant missing")


@pytest.mark.parametrize("dist", ["uniform", "int"])
def test_grouped_matches_oracle_and_single_launches(dist):
    import paper_1609_00076_amd as mdg
    import torch
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = _batch(1 if dist == "uniform" else 2, 120, 1, 300, dist=dist, special=True)
    gemms = _to_device(probs)
    classes = [i % 2 for i in range(len(gemms))]
    plan = GroupedPlan(gemms, classes, mdg.MDG_SCHEDULE_LPT)
    plan.launch()
    torch.cuda.synchronize()
    _check_against_oracle(probs, gemms, exact=(dist == "int"))
    # the same GEMMs one by one with the variant of their tile class: bitwise equal
    for p, g, c in zip(probs, gemms, classes):
        dC = torch.from_numpy(p["C"]).cuda()
        st = mdg.mdg_dgemm_ex(_variant_of_class(c), p["transa"], p["transb"], p["m"], p["n"],
                              p["k"], p["alpha"], g["A"], p["lda"], g["B"], p["ldb"], p["beta"],
                              dC, p["ldc"])
        assert st == 0
        torch.cuda.synchronize()
        assert same_bits(dC.cpu().numpy(), g["C"].cpu().numpy())


@pytest.mark.parametrize("dist", ["uniform", "int"])
def test_wave_plan_matches_oracle_and_single_launches(dist):
    """Class 2 (every GEMM on 32x32 wave tiles): each GEMM matches the oracle (bit-exact on
    integers), and is bitwise the single-GEMM wave variant's result and a ring variant's (the same
    k-order), on the default grid and on grids that make waves walk many tiles."""
    import paper_1609_00076_amd as mdg
    import torch
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = _batch(5 if dist == "uniform" else 6, 150, 1, 300, dist=dist, special=True)
    ring = [v for v in range(mdg.mdg_num_variants())
            if mdg.mdg_variant_name(v) == "ring_f64_128x64x16_w32x32_s3_il"][0]
    alone = {}
    for name, v in (("wave", _variant_of_class(2)), ("ring", ring)):
        outs = []
        for p in probs:
            dA, dB = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
            dC = torch.from_numpy(p["C"]).cuda()
            assert mdg.mdg_dgemm_ex(v, p["transa"], p["transb"], p["m"], p["n"], p["k"],
                                    p["alpha"], dA, p["lda"], dB, p["ldb"], p["beta"], dC,
                                    p["ldc"]) == 0
            outs.append(dC)
        torch.cuda.synchronize()
        alone[name] = [o.cpu().numpy() for o in outs]
    for sched, grid in ((mdg.MDG_SCHEDULE_LPT, 0), (mdg.MDG_SCHEDULE_NATURAL, 8),
                        (mdg.MDG_SCHEDULE_LPT, 24)):
        gemms = _to_device(probs)
        GroupedPlan(gemms, [2] * len(gemms), sched).launch(grid)
        torch.cuda.synchronize()
        _check_against_oracle(probs, gemms, exact=(dist == "int"))
        for i, g in enumerate(gemms):
            got = g["C"].cpu().numpy()
            assert same_bits(got, alone["wave"][i]), f"GEMM {i}: grouped vs single wave launch"
            assert same_bits(got, alone["ring"][i]), f"GEMM {i}: grouped vs ring variant"


def test_schedules_and_grids_agree_bitwise():
    import paper_1609_00076_amd as mdg
    import torch
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = _batch(3, 60, 16, 200)
    outs = []
    for sched, grid in ((mdg.MDG_SCHEDULE_NATURAL, 0), (mdg.MDG_SCHEDULE_LPT, 7),
                        (mdg.MDG_SCHEDULE_LPT, 2048)):
        gemms = _to_device(probs)
        GroupedPlan(gemms, None, sched).launch(grid)
        torch.cuda.synchronize()
        outs.append([g["C"].cpu().numpy() for g in gemms])
    for o in outs[1:]:
        assert all(same_bits(a, b2) for a, b2 in zip(o, outs[0]))


def test_graph_replays():
    import paper_1609_00076_amd as mdg
    import torch
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = _batch(4, 80, 8, 256, special=True)
    gemms = _to_device(probs)
    c0 = [g["C"].clone() for g in gemms]
    plan = GroupedPlan(gemms, None, mdg.MDG_SCHEDULE_LPT)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.launch()  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch()
    side = synth.problem(41, 0, "N", "N", 300, 200, 100)
    dA, dB, dC = (torch.from_numpy(side[x]).cuda() for x in "ABC")
    for replay in range(3):
        for g, c in zip(gemms, c0):
            g["C"].copy_(c)
        # unrelated eager work between replays
        assert mdg.mdg_dgemm("N", "N", 300, 200, 100, 1.0, dA, side["lda"], dB, side["ldb"], 0.5,
                             dC, side["ldc"]) == 0
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check_against_oracle(probs, gemms, exact=False)


def test_full_batch_graph_replays_match_oracle():
    """The benchmark's batch itself: 2048 GEMMs with m, n, k log-uniform in [16, 512], random
    transposes and scalars, tight leading dimensions, under the tuned policy. One grouped launch is
    captured in a graph and replayed twice (C reset between replays), on the tuned grid and on the
    default grid (where each workgroup walks several tiles); every GEMM is compared with the
    oracle element by element at 1e-13 of D, and its C padding must stay untouched."""
    import torch
    from paper_1609_00076_amd import tuner
    from paper_1609_00076_amd.grouped import GroupedPlan
    probs = synth.grouped_batch()
    assert len(probs) == 2048
    refs = [run_oracle(p, p["alpha"], p["beta"]) for p in probs]
    gemms = _to_device(probs)
    c0 = [g["C"].clone() for g in gemms]
    tuned = tuner.best_policy(tuner.GROUPED_SIGNATURE)
    wave = {"tile": "wave", "threshold": 0, "schedule": 1, "grid": 0}
    for policy, grid in ((tuned, tuned["grid"]), (tuned, 0), (wave, 0)):
        plan = GroupedPlan(gemms, tuner.classes_for(gemms, policy), policy["schedule"])
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.launch(grid)  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.launch(grid)
        for replay in range(2):
            for g, c in zip(gemms, c0):
                g["C"].copy_(c)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            print(f"[grouped] 2048-GEMM batch, policy {policy}, grid {grid}, replay {replay}: "
                  "checking", flush=True)
            worst = 0.0
            for i, (p, g, (ref, D)) in enumerate(zip(probs, gemms, refs)):
                got = g["C"].cpu().numpy()
                m, n, ldc = p["m"], p["n"], p["ldc"]
                e = rel_err(logical(got, m, n, ldc).T, logical(ref, m, n, ldc).T, D)
                worst = max(worst, e)
                assert e <= TOL, f"GEMM {i} {p['transa']}{p['transb']} {m}x{n}x{p['k']}: {e:.2e}"
                if ldc > m:
                    assert np.all(got.view(np.uint64).reshape(n, ldc)[:, m:] == synth.PAD_C_BITS)
            print(f"[grouped] worst error {worst:.2e}", flush=True)

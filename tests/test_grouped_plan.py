"""Grouped-launch plans on the CPU: the plan builder is host-only and dereferences nothing."""
import struct

import numpy as np
import pytest

import paper_1609_00076_amd as mdg
from paper_1609_00076_amd import binding as b

FAKE = 0x10000  # addresses are only stored, never dereferenced by the plan builder


def _desc(ta="N", tb="N", m=70, n=40, k=30, alpha=1.0, beta=0.5, lda=None, ldb=None, ldc=None):
    lda = lda or max(1, m if ta == "N" else k)
    ldb = ldb or max(1, k if tb == "N" else n)
    ldc = ldc or max(1, m)
    return b.mdg_gemm_desc(ta.encode(), tb.encode(), m, n, k, alpha, FAKE, lda, FAKE, ldb, beta,
                           FAKE, ldc)


def _plan(descs, classes=None, schedule=mdg.MDG_SCHEDULE_LPT):
    nbytes = mdg.mdg_grouped_plan_bytes(descs, classes)
    buf = np.zeros(nbytes, dtype=np.uint8)
    st, nt, bad = mdg.mdg_grouped_plan(descs, classes, schedule, buf)
    return st, nt, bad, buf


def _tiles(buf, kind=0):
    magic, version, count, k, ntiles, doff, toff = struct.unpack_from("<iiiiqqq", buf, 0)
    assert magic == 0x4D444750 and version == 2 and k == kind
    return count, np.frombuffer(buf[toff:toff + 16 * ntiles], dtype=np.int32).reshape(-1, 4), doff


def test_every_tile_once_and_lpt_order():
    rng = np.random.default_rng(1)
    descs, classes = [], []
    for _ in range(60):
        m, n, k = (int(x) for x in rng.integers(1, 300, 3))
        descs.append(_desc("NT"[rng.integers(2)], "NT"[rng.integers(2)], m, n, k))
        classes.append(int(rng.integers(2)))
    st, nt, bad, buf = _plan(descs, classes)
    assert st == 0 and bad == -1
    count, tiles, _ = _tiles(buf)
    assert count == 60 and len(tiles) == nt
    want = set()
    for i, (d, c) in enumerate(zip(descs, classes)):
        t = 64 if c == 0 else 32
        for tn in range(-(-d.n // t)):
            for tm in range(-(-d.m // t)):
                want.add((i, tm, tn))
    got = [tuple(int(x) for x in row[:3]) for row in tiles]
    assert len(got) == len(set(got)) and set(got) == want
    cost = [(64 if classes[g] == 0 else 32) ** 2 * descs[g].k for g, _, _ in got]
    assert all(a >= b2 for a, b2 in zip(cost, cost[1:])), "LPT order"


def test_natural_order_and_automatic_classes():
    descs = [_desc(m=100, n=20), _desc(m=130, n=130), _desc(m=47, n=47)]
    st, nt, _, buf = _plan(descs, None, mdg.MDG_SCHEDULE_NATURAL)
    assert st == 0
    _, tiles, _ = _tiles(buf)
    # automatic: class 1 (32x32) when m < 48 or n < 48
    assert nt == 4 * 1 + 3 * 3 + 2 * 2  # 100x20 -> 32x32 tiles: 4x1; 130x130 -> 64: 3x3; 47x47 -> 32: 2x2
    assert list(tiles[:, 0]) == sorted(tiles[:, 0])


def test_quick_returns_have_no_tiles_but_scaling_does():
    descs = [_desc(m=0), _desc(n=0), _desc(alpha=0.0, beta=1.0), _desc(k=0, beta=1.0, lda=70),
             _desc(alpha=0.0, beta=2.0), _desc(k=0, beta=0.0, lda=70)]
    st, nt, _, buf = _plan(descs, [0] * 6)
    assert st == 0
    _, tiles, _ = _tiles(buf)
    assert sorted(set(int(g) for g in tiles[:, 0])) == [4, 5]


def test_invalid_gemm_reports_index_and_code():
    descs = [_desc(), _desc(), _desc(m=50, ldc=10)]
    nbytes = mdg.mdg_grouped_plan_bytes(descs, None)
    buf = np.zeros(nbytes, dtype=np.uint8)
    st, _, bad = mdg.mdg_grouped_plan(descs, None, mdg.MDG_SCHEDULE_LPT, buf)
    assert st == 113 and bad == 2
    assert mdg.mdg_grouped_plan(descs[:2], None, 7, buf)[0] == 4
    assert mdg.mdg_grouped_plan_bytes(descs, [0, 1, 5]) == -1
    small = np.zeros(16, dtype=np.uint8)
    assert mdg.mdg_grouped_plan(descs[:2], None, mdg.MDG_SCHEDULE_LPT, small)[0] == 5


def test_descriptor_contents():
    d = _desc("T", "N", m=33, n=21, k=17, alpha=-2.0, beta=0.25, lda=20, ldb=19, ldc=40)
    st, _, _, buf = _plan([d], [1])
    assert st == 0
    _, _, doff = _tiles(buf)
    m, n, k, lda, ldb, ldc = struct.unpack_from("<6q", buf, doff)
    alpha, beta = struct.unpack_from("<2d", buf, doff + 48)
    a, bb, c, ext_a, ext_b = struct.unpack_from("<3Q2q", buf, doff + 64)
    ta, tb, cls, tiles_m, tiles_n = struct.unpack_from("<5i", buf, doff + 104)
    assert (m, n, k, lda, ldb, ldc) == (33, 21, 17, 20, 19, 40)
    assert (alpha, beta) == (-2.0, 0.25) and (a, bb, c) == (FAKE, FAKE, FAKE)
    assert ext_a == (33 - 1) * 20 + 17 and ext_b == (21 - 1) * 19 + 17  # A stored k x m, B k x n
    assert (ta, tb, cls, tiles_m, tiles_n) == (1, 0, 1, 2, 1)


def test_launch_argument_checks_return_before_any_device_call():
    assert mdg.mdg_dgemm_grouped(None, 5) == 1
    assert mdg.mdg_dgemm_grouped(FAKE + 8, 5) == 1  # misaligned
    assert mdg.mdg_dgemm_grouped(FAKE, -1) == 2
    assert mdg.mdg_dgemm_grouped(FAKE, 5, grid=-3) == 3
    assert mdg.mdg_dgemm_grouped(FAKE, 0) == 0
    assert mdg.mdg_grouped_tile_classes() == 3


def _wave_batch(count=90, seed=3):
    rng = np.random.default_rng(seed)
    descs = []
    for _ in range(count):
        m, n, k = (int(x) for x in rng.integers(1, 400, 3))
        descs.append(_desc("NT"[rng.integers(2)], "NT"[rng.integers(2)], m, n, k))
    return descs


@pytest.mark.parametrize("schedule", [mdg.MDG_SCHEDULE_LPT, mdg.MDG_SCHEDULE_NATURAL])
def test_wave_plan_xcd_sublists(schedule):
    """Wave-tile plans (class 2 for every GEMM): every 32x32 tile exactly once; the tile list is cut
    into 8 XCD sublists (offsets after the header), each GEMM wholly in one sublist with its tiles
    contiguous and column by column; LPT gives GEMMs to XCDs by decreasing cost to the least loaded
    one (so no XCD ends with more than the lightest plus the largest GEMM), NATURAL round-robin."""
    descs = _wave_batch()
    st, nt, bad, buf = _plan(descs, [2] * len(descs), schedule)
    assert st == 0 and bad == -1
    count, tiles, doff = _tiles(buf, kind=1)
    assert doff == 64 + 80
    xoff = struct.unpack_from("<9q", buf, 64)
    assert xoff[0] == 0 and xoff[8] == nt == len(tiles) and list(xoff) == sorted(xoff)
    want = {(i, tm, tn) for i, d in enumerate(descs)
            for tn in range(-(-d.n // 32)) for tm in range(-(-d.m // 32))}
    got = [tuple(int(x) for x in row[:3]) for row in tiles]
    assert len(got) == len(set(got)) and set(got) == want
    owner, load = {}, [0.0] * 8
    for x in range(8):
        sub = got[xoff[x]:xoff[x + 1]]
        seen = []
        for g, tm, tn in sub:
            assert owner.setdefault(g, x) == x, "a GEMM split over XCDs"
            if not seen or seen[-1] != g:
                assert g not in seen, "a GEMM's tiles not contiguous"
                seen.append(g)
        for g in seen:
            gt = [(tm, tn) for gg, tm, tn in sub if gg == g]
            assert gt == sorted(gt, key=lambda t: (t[1], t[0])), "column by column"
            load[x] += len(gt) * 32 * 32 * descs[g].k
    cost = {g: -(-descs[g].m // 32) * -(-descs[g].n // 32) * 1024 * descs[g].k for g in owner}
    if schedule == mdg.MDG_SCHEDULE_LPT:
        assert max(load) - min(load) <= max(cost.values())
    else:
        assert all(owner[g] == i % 8 for i, g in enumerate(sorted(owner)))


def test_wave_class_cannot_mix_with_workgroup_classes():
    descs = _wave_batch(10)
    assert mdg.mdg_grouped_plan_bytes(descs, [2] * 9 + [0]) == -1
    buf = np.zeros(1 << 16, dtype=np.uint8)
    assert mdg.mdg_grouped_plan(descs, [2] * 9 + [1], mdg.MDG_SCHEDULE_LPT, buf)[0] == 3
    n0 = mdg.mdg_grouped_plan_bytes(descs, [2] * 10)
    tiles = sum(-(-d.m // 32) * -(-d.n // 32) for d in descs)
    assert n0 == 64 + 80 + 10 * 136 + 16 * tiles  # 136-byte descriptors


def test_tuner_times_each_candidate_with_its_own_tile_kind(monkeypatch):
    """The tuner builds each candidate's plan with that candidate's tile classes (wave tiles for a
    wave policy, the threshold's workgroup classes otherwise); the plan constructor is replaced
    by a recorder, so nothing reaches the GPU."""
    from paper_1609_00076_amd import tuner
    seen = []

    class Stop(Exception):
        pass

    def fake_plan(gemms, classes, schedule):
        seen.append((list(classes), schedule))
        raise Stop

    monkeypatch.setattr(tuner, "GroupedPlan", fake_plan)
    gemms = [dict(m=m, n=n) for m, n in ((30, 100), (100, 100), (50, 39))]
    for pol, want in (({"tile": "wave", "threshold": 0, "schedule": 1, "grid": 512}, [2, 2, 2]),
                      ({"tile": "block", "threshold": 40, "schedule": 0, "grid": 512}, [1, 0, 1]),
                      ({"tile": "block", "threshold": 0, "schedule": 1, "grid": 256}, [0, 0, 0])):
        with pytest.raises(Stop):
            tuner.time_policy(gemms, pol)
        assert seen[-1] == (want, pol["schedule"])

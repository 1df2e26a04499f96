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


def _tiles(buf):
    magic, version, count, _, ntiles, doff, toff = struct.unpack_from("<iiiiqqq", buf, 0)
    assert magic == 0x4D444750 and version == 1
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
    assert mdg.mdg_grouped_tile_classes() == 2

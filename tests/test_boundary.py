"""The C-ABI boundary on the CPU: symbols, argument checks, quick returns, host helpers.

No call here reaches a kernel: every call either fails an argument check or is a
quick return, both of which return before any HIP call.
"""
import os
import re

import pytest

import paper_1609_00076_amd as mdg
from paper_1609_00076_amd.build import INCLUDE, LIB_PATH

HEADER = os.path.join(INCLUDE, "mdg.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mdg_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mdg.load()  # the binding's loader (torch's HIP runtime first)
    assert lib._name == LIB_PATH
    names = _declared_functions()
    assert "mdg_dgemm" in names and len(names) >= 8
    for name in names:
        assert hasattr(lib, name), f"{name} declared in mdg.h but not exported"
        assert hasattr(mdg, name), f"{name} has no Python binding of the same name"


def test_version_and_variants():
    assert mdg.mdg_version() >= 100
    nv = mdg.mdg_num_variants()
    assert nv >= 2
    names = [mdg.mdg_variant_name(v) for v in range(nv)]
    assert all(names) and len(set(names)) == nv
    assert mdg.mdg_variant_name(nv) is None and mdg.mdg_variant_name(-1) is None
    for v in range(nv):
        mt, nt, kt, threads = mdg.mdg_variant_info(v)
        assert mt % 16 == 0 and nt % 16 == 0 and kt % 4 == 0 and threads % 64 == 0
    with pytest.raises(mdg.MdgError):
        mdg.mdg_variant_info(nv)


def _call(ta="N", tb="N", m=4, n=4, k=4, alpha=1.0, A=0x1000, lda=4, B=0x1000, ldb=4,
          beta=0.0, C=0x1000, ldc=4, variant=None):
    # Fake non-NULL addresses: every case below fails an argument check or returns early,
    # so none of them is ever dereferenced.
    args = (ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc)
    if variant is None:
        return mdg.mdg_dgemm(*args)
    return mdg.mdg_dgemm_ex(variant, *args)


@pytest.mark.parametrize("kw,code", [
    (dict(ta="X"), 1), (dict(ta=""), 1), (dict(tb="q"), 2),
    (dict(m=-1), 3), (dict(n=-2), 4), (dict(k=-3), 5),
    (dict(A=None), 7), (dict(lda=3), 8), (dict(ta="T", m=4, k=8, lda=4), 8),
    (dict(B=None), 9), (dict(ldb=3), 10), (dict(tb="t", n=8, ldb=4), 10),
    (dict(C=None), 12), (dict(ldc=3), 13),
    (dict(ta="X", m=-1, lda=0), 1), (dict(m=-1, lda=0), 3),  # first bad argument wins
    (dict(m=0, lda=0), 8), (dict(n=0, ldc=0), 13),  # ld >= 1 even for empty matrices
])
def test_argument_codes(kw, code):
    assert _call(**kw) == code
    assert mdg.mdg_status_string(code).startswith(f"invalid argument {code}")


def test_null_allowed_where_not_dereferenced_and_quick_returns():
    # m == 0 or n == 0: nothing touched, NULL everywhere is fine
    assert _call(m=0, A=None, B=None, C=None, lda=1, ldc=1) == 0
    assert _call(n=0, A=None, B=None, C=None) == 0
    # alpha == 0 (or k == 0) with beta == 1: quick return, nothing read
    assert _call(alpha=0.0, beta=1.0, A=None, B=None, C=None) == 0
    assert _call(k=0, beta=1.0, A=None, B=None, C=None, lda=4, ldb=1) == 0
    # alpha == 0 with beta != 1 still needs C (A, B may stay NULL)
    assert _call(alpha=0.0, beta=2.0, A=None, B=None, C=None) == 12


def test_variant_errors():
    assert _call(variant=mdg.mdg_num_variants(), m=0) == -2
    assert _call(variant=-7, m=0) == -2
    assert _call(variant=0, m=-1) == 3  # argument checks come first
    assert mdg.mdg_status_string(-2) == "unknown kernel variant"
    assert mdg.mdg_status_string(12345) == "unknown status"


def test_select_variant_is_pure_host_logic():
    nv = mdg.mdg_num_variants()
    assert mdg.mdg_select_variant("N", "N", 0, 4, 4, 1.0, 0.0) == -1
    assert mdg.mdg_select_variant("N", "N", 4, 4, 4, 0.0, 0.5) == -1
    assert mdg.mdg_select_variant("N", "X", 4, 4, 4, 1.0, 0.0) == -1
    for shape in [(256, 256, 256), (8192, 8192, 8192), (4099, 4099, 4099), (8192, 8192, 64)]:
        for ta in "NT":
            for tb in "NT":
                v = mdg.mdg_select_variant(ta, tb, *shape, 1.0, 1.0)
                assert 0 <= v < nv


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1609_00076_amd.binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        b.mdg_version()


def test_leading_dimension_offset_guard_is_host_side_and_exact():
    """The panel-offset guard refuses only what the 32-bit panel offsets cannot address, and it
    does so on the host, before any HIP call (raw addresses: nothing is dereferenced)."""
    big = 1 << 28   # 2^28 elements: two such rows of a panel already span 4 GiB of bytes
    fake = 1 << 40  # never dereferenced
    # op(A) = A^T stored k x m: 300 rows of op(A) strided by lda
    st = mdg.mdg_dgemm("T", "N", 300, 64, 64, 1.0, fake, big, fake, 64, 0.0, fake, 300)
    assert st == -4, mdg.mdg_status_string(st)
    # A stored m x k: 64 k-columns strided by lda
    st = mdg.mdg_dgemm("N", "N", 64, 64, 64, 1.0, fake, big, fake, 64, 0.0, fake, 64)
    assert st == -4
    # op(B) columns strided by ldb (B stored k x n)
    st = mdg.mdg_dgemm("N", "N", 64, 300, 64, 1.0, fake, 64, fake, big, 0.0, fake, 64)
    assert st == -4
    # one row and one k-index: nothing inside the matrix is more than one element away, so the
    # guard lets it through (here the call then stops at the device check: no GPU)
    st = mdg.mdg_dgemm("T", "T", 1, 1, 1, 1.0, fake, big, fake, big, 0.0, fake, 1)
    assert st != -4 and st < 0
    # a C of 40 million rows and one column: too many thin-kernel workgroups for one launch, so
    # the product stays on the tiles, whose grid fits (the call then stops at the device check)
    st = mdg.mdg_dgemm("N", "N", 40_000_000, 1, 1, 1.0, fake, 40_000_000, fake, 1, 0.0, fake,
                       40_000_000)
    assert st != -4 and st < 0
    # alpha = 0: A and B are not read, so their leading dimensions do not matter
    st = mdg.mdg_dgemm("T", "N", 300, 64, 64, 0.0, fake, big, fake, 64, 1.0, fake, 300)
    assert st == 0  # quick return (beta = 1)


def test_sweep_variant_choice():
    """The measured choice for the sweep shapes (each a variant whose efficiency was measured on the
    GPU for that transpose case): 256x128 or 128x256 ring tiles from 4096 up (4099 on its 4096
    block), the k-split 128x128 ring tile for 2048 and the k-split 64x64 one for 1024 (one tile per
    CU), the register-staged 128x64 tile for the HBM-bound k = 64 case."""
    def name(ta, tb, m, n, k):
        return mdg.mdg_variant_name(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0))
    want = {"NN": "ring_f64_128x256x16_w128x32_s3_il", "NT": "ring_f64_128x256x16_w64x64_s3_il",
            "TN": "ring_f64_256x128x16_w128x32_s3_il", "TT": "ring_f64_256x128x16_w64x64_s3_il"}
    for size in (4096, 8192, 16384):
        for ta in "NT":
            for tb in "NT":
                assert name(ta, tb, size, size, size) == want[ta + tb]
    for ta in "NT":
        for tb in "NT":
            assert name(ta, tb, 1024, 1024, 1024) == "ringk2_f64_64x64x16_w32x32_s4"
            assert name(ta, tb, 2048, 2048, 2048) == "ringk2_f64_128x128x16_w64x64_s2"
            assert name(ta, tb, 8192, 8192, 64) == "mfma_f64_128x64x16_w32x32"


def test_dgemm_plan_splits_off_thin_fringes():
    """A fringe of at most 16 rows or columns left by the big tiles goes to the thin kernel; the
    tiled block takes the variant of the divisible size. Thin products go to the thin kernel
    alone; sizes the big tiles divide are not split."""
    plan = mdg.mdg_dgemm_plan
    for ta in "NT":
        for tb in "NT":
            whole = mdg.mdg_select_variant(ta, tb, 4096, 4096, 4096, 1.0, 1.0)
            assert plan(ta, tb, 4096, 4096, 4096) == (whole, 4096, 4096)
            for size in (4097, 4099, 4112):
                v, m0, n0 = plan(ta, tb, size, size, size)
                assert (v, m0, n0) == (whole, 4096, 4096), (ta, tb, size)
                assert mdg.mdg_select_variant(ta, tb, size, size, size, 1.0, 1.0) == v
            assert plan(ta, tb, 4113, 4113, 4113)[1:] == (4113, 4113)  # fringe of 17: no split
            for m, n, k in ((3, 4099, 4099), (4099, 3, 4099), (16, 5000, 300), (1, 1, 4000)):
                assert plan(ta, tb, m, n, k) == (-1, 0, 0)
                assert mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0) == -1
    for args, pos in ((("X", "N", 4, 4, 4), 1), (("N", "Y", 4, 4, 4), 2), (("N", "N", 0, 4, 4), 3),
                      (("N", "N", 4, -1, 4), 4), (("N", "N", 4, 4, 0), 5)):
        with pytest.raises(mdg.MdgError) as e:
            plan(*args)
        assert e.value.status == pos


def test_every_variant_is_reachable():
    """No dead entries in the kernel table: each variant is the automatic choice for some shape and
    transpose case, a grouped tile class, or a dsyrk configuration."""
    import numpy as np
    nv = mdg.mdg_num_variants()
    sizes = sorted({int(x) for x in np.round(np.logspace(0, 4.3, 60))})
    chosen = set()
    for ta in "NT":
        for tb in "NT":
            for m in sizes:
                for n in sizes:
                    for k in (16, 64, 256, 257, 1024, 2048, 8192):
                        chosen.add(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0))
            for n in sizes:
                for k in (64, 1024, 8192):
                    for uplo in "LU":
                        chosen.add(mdg.mdg_dsyrk_select_variant(uplo, ta, n, k))
    grouped = {"mfma_f64_64x64x16_w32x32", "mfma_f64_32x32x16_w16x16", "wave_f64_64x64x8_w32x32"}
    for v in range(nv):
        name = mdg.mdg_variant_name(v)
        assert v in chosen or name in grouped, f"variant {v} ({name}) is never used"


def test_single_round_grids_take_the_k_split_tile():
    """A grid of at most one 64x64 tile per CU (256 CUs) with k above the short-k bound runs the
    k-split configuration of that tile: two groups up to k = 2048, four beyond; more tiles or short
    k keep the one-group choice. One round of 128x128 tiles that fills most of the GPU runs the
    k-split 128x128 tile."""
    name = mdg.mdg_variant_name
    for ta in "NT":
        for tb in "NT":
            for m, n, k in ((1024, 1024, 1024), (1000, 1000, 300), (1024, 1024, 2048)):
                assert name(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0)) == \
                    "ringk2_f64_64x64x16_w32x32_s4"
            for m, n, k in ((512, 2048, 4096), (1024, 1024, 2049), (1024, 1024, 8192)):
                assert name(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0)) == \
                    "ringk4_f64_64x64x16_w32x32_s2"
            for m, n, k in ((1024, 1024, 256), (1089, 1024, 1024), (1536, 1536, 2048),
                            (8192, 8192, 8192)):
                assert not name(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0)).startswith("ringk")
            for m, n, k in ((2048, 2048, 2048), (2048, 2048, 8192), (642, 4924, 4096)):
                assert name(mdg.mdg_select_variant(ta, tb, m, n, k, 1.0, 1.0)) == \
                    "ringk2_f64_128x128x16_w64x64_s2"


# ---- level-3 entry points: checks and refusals that return before any HIP call ----------------

FAKE = 0x1000  # a non-NULL address that none of the cases below dereferences


def _syrk(uplo="L", trans="N", n=4, k=4, alpha=1.0, A=FAKE, lda=4, beta=0.5, C=FAKE, ldc=4,
          variant=None):
    args = (uplo, trans, n, k, alpha, A, lda, beta, C, ldc)
    return mdg.mdg_dsyrk(*args) if variant is None else mdg.mdg_dsyrk_ex(variant, *args)


@pytest.mark.parametrize("kw,code", [
    (dict(uplo="X"), 1), (dict(trans="Q"), 2), (dict(n=-1), 3), (dict(k=-1), 4),
    (dict(A=None), 6), (dict(lda=3), 7), (dict(trans="T", n=4, k=8, lda=4), 7),
    (dict(C=None), 9), (dict(ldc=3), 10), (dict(uplo="X", n=-1), 1),
])
def test_dsyrk_argument_codes(kw, code):
    assert _syrk(**kw) == code


def test_dsyrk_quick_returns_and_refusals():
    assert _syrk(n=0, A=None, C=None, lda=1, ldc=1) == 0
    assert _syrk(alpha=0.0, beta=1.0, A=None, C=None) == 0
    assert _syrk(k=0, beta=1.0, A=None, C=None) == 0
    assert _syrk(variant=mdg.mdg_num_variants()) == -2
    names = [mdg.mdg_variant_name(v) for v in range(mdg.mdg_num_variants())]
    assert _syrk(variant=names.index("mfma_f64_64x64x16_w32x32")) == -2  # no ring tile
    # a k-panel of A would span 4 GiB of 32-bit offsets: refused on the host
    assert _syrk(n=4, k=100, lda=600_000_000) == -4


def test_dsyrk_choice_is_host_logic():
    # n = 8192 splits: the triangle launch covers eight diagonal blocks of order 1024, on 64x64
    # tiles; n = 6144 is one launch over the whole triangle, on 128x64 tiles
    vid = mdg.mdg_dsyrk_select_variant("L", "N", 8192, 8192)
    assert mdg.mdg_variant_name(vid) == "ring_f64_64x64x16_w32x32_s3_il"
    vid = mdg.mdg_dsyrk_select_variant("L", "N", 6144, 6144)
    assert mdg.mdg_variant_name(vid) == "ring_f64_128x64x16_w32x32_s3_il"
    # the split needs k >= 2048: below it n = 8192 is one launch over the whole triangle
    assert mdg.mdg_variant_name(mdg.mdg_dsyrk_select_variant("L", "N", 8192, 2048)) == \
        "ring_f64_64x64x16_w32x32_s3_il"
    assert mdg.mdg_variant_name(mdg.mdg_dsyrk_select_variant("L", "N", 8192, 2047)) == \
        "ring_f64_128x64x16_w32x32_s3_il"

    for uplo, trans in (("U", "N"), ("L", "T"), ("U", "T")):
        assert mdg.mdg_dsyrk_select_variant(uplo, trans, 8192, 8192) >= 0
    assert mdg.mdg_dsyrk_select_variant("X", "N", 10, 10) == -2
    assert mdg.mdg_dsyrk_select_variant("L", "N", -1, 10) == -2


def _tri(name, side="L", uplo="L", transa="N", diag="N", m=4, n=4, alpha=1.0, A=FAKE, lda=4,
         B=FAKE, ldb=4):
    return getattr(mdg, name)(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb)


@pytest.mark.parametrize("name", ["mdg_dtrmm", "mdg_dtrsm"])
@pytest.mark.parametrize("kw,code", [
    (dict(side="X"), 1), (dict(uplo="X"), 2), (dict(transa="X"), 3), (dict(diag="X"), 4),
    (dict(m=-1), 5), (dict(n=-1), 6), (dict(A=None), 8), (dict(lda=3), 9),
    (dict(side="R", m=4, n=8, lda=4), 9), (dict(side="R", m=8, n=4, lda=4, ldb=8), 0),
    (dict(B=None), 10), (dict(ldb=3), 11), (dict(side="X", m=-1), 1),
])
def test_tri_argument_codes(name, kw, code):
    if code == 0:
        # valid arguments would launch kernels: check the same case with m = 0 instead
        kw = dict(kw, m=0)
    assert _tri(name, **kw) == code


@pytest.mark.parametrize("name", ["mdg_dtrmm", "mdg_dtrsm"])
def test_tri_plans_are_checked_before_any_launch(name):
    assert _tri(name, m=0, A=None, B=None) == 0
    assert _tri(name, n=0, A=None, B=None) == 0
    # m = 300 needs GEMMs on submatrices; with ldb this large a k-panel of B's 200 columns
    # would span 4 GiB of 32-bit offsets, so the whole call is refused before anything is enqueued
    assert _tri(name, m=300, n=200, lda=300, ldb=40_000_000) == -4


@pytest.mark.parametrize("kw,code", [
    (dict(ta="X"), 1), (dict(tb="q"), 2), (dict(m=-1), 3), (dict(n=-2), 4), (dict(k=-3), 5),
    (dict(A=None), 7), (dict(lda=3), 8), (dict(B=None), 9), (dict(ldb=3), 10),
    (dict(C=None), 12), (dict(ldc=3), 13), (dict(S=0), 14), (dict(S=11), 14),
])
def test_split_noalloc_argument_codes(kw, code):
    """The no-allocation split entry point checks arguments as mdg_dgemm_split does (fake
    addresses, never dereferenced: each call fails a check before any HIP call)."""
    a = dict(ta="N", tb="N", m=4, n=4, k=4, alpha=1.0, A=0x1000, lda=4, B=0x1000, ldb=4, beta=0.0,
             C=0x1000, ldc=4, S=7)
    a.update(kw)
    st = mdg.mdg_dgemm_split_noalloc(a["ta"], a["tb"], a["m"], a["n"], a["k"], a["alpha"], a["A"],
                                     a["lda"], a["B"], a["ldb"], a["beta"], a["C"], a["ldc"],
                                     a["S"])
    assert st == code


def test_split_noalloc_scratch_limit_is_host_side():
    """Problems whose workspace exceeds the static scratch array are refused with MDG_ERR_SCRATCH
    before any HIP call; quick returns need no scratch."""
    cap = mdg.mdg_dgemm_split_noalloc_max_bytes()
    assert cap == 64 << 20
    fake = 1 << 40
    assert mdg.mdg_dgemm_split_workspace_size(2048, 2048, 2048, 7) <= cap
    assert mdg.mdg_dgemm_split_workspace_size(2048, 2048, 2048, 8) > cap
    st = mdg.mdg_dgemm_split_noalloc("N", "N", 2048, 2048, 2048, 1.0, fake, 2048, fake, 2048, 0.0,
                                     fake, 2048, 8)
    assert st == mdg.MDG_ERR_SCRATCH
    assert "scratch" in mdg.mdg_status_string(st)
    # a problem that fits passes the limit and stops at the device check here (no GPU)
    st = mdg.mdg_dgemm_split_noalloc("N", "N", 2048, 2048, 2048, 1.0, fake, 2048, fake, 2048, 0.0,
                                     fake, 2048, 7)
    assert st in (mdg.MDG_ERR_HIP, mdg.MDG_ERR_DEVICE)
    assert mdg.mdg_dgemm_split_noalloc("N", "N", 0, 5, 5, 1.0, None, 1, None, 5, 0.0, None, 1,
                                       7) == 0
    assert mdg.mdg_dgemm_split_noalloc("N", "N", 5, 5, 5, 0.0, None, 5, None, 5, 1.0, None, 5,
                                       7) == 0


def test_split_entry_points_check_the_device_after_the_arguments():
    """Argument and size checks come first; then, before any launch, the device check (on this
    CPU-only host it fails with a runtime code rather than launching)."""
    fake = 1 << 40
    need = mdg.mdg_dgemm_split_workspace_size(64, 64, 64, 7)
    st = mdg.mdg_dgemm_split("N", "N", 64, 64, 64, 1.0, fake, 64, fake, 64, 0.0, fake, 64, 7,
                             fake, need)
    assert st in (mdg.MDG_ERR_HIP, mdg.MDG_ERR_DEVICE)
    assert mdg.mdg_dgemm_split("N", "N", 64, 64, 64, 1.0, fake, 64, fake, 64, 0.0, fake, 64, 7,
                               fake, need - 1) == 15
    st = mdg.mdg_split_slices(0, "N", 64, 64, fake, 64, 7, fake, fake)
    assert st in (mdg.MDG_ERR_HIP, mdg.MDG_ERR_DEVICE)
    assert mdg.mdg_split_slices(0, "N", 64, 64, fake, 63, 7, fake, fake) == 6


def test_crt_bits_and_workspace_are_host_logic():
    import oracle.ozaki as oz
    for nmod in range(1, mdg.mdg_crt_max_moduli() + 1):
        for k in (0, 1, 7, 32, 1000, 8192, 140000):
            assert mdg.mdg_crt_bits(k, nmod) == oz.crt_bits(k, nmod), (k, nmod)
    assert mdg.mdg_crt_bits(100, 0) == 0 and mdg.mdg_crt_bits(100, 25) == 0
    assert tuple(oz.MODULI) == (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199,
                                197, 193, 191, 181, 179, 173, 167, 163, 157, 151, 149)
    rnd = lambda x, a: -(-x // a) * a  # noqa: E731
    m, n, k, N = 300, 190, 70, 15
    want = (rnd(N * 384 * 128, 256) + rnd(N * 256 * 128, 256) + rnd(N * m * rnd(n, 4), 256)
            + rnd(4 * m, 256) + rnd(4 * n, 256))
    assert mdg.mdg_dgemm_crt_workspace_size(m, n, k, N) == want
    assert mdg.mdg_dgemm_crt_workspace_size(m, n, k, 0) == -1
    fake = 1 << 40
    st = mdg.mdg_dgemm_crt("N", "N", 64, 64, 64, 1.0, fake, 64, fake, 64, 0.0, fake, 64, 15, fake,
                           mdg.mdg_dgemm_crt_workspace_size(64, 64, 64, 15))
    assert st in (mdg.MDG_ERR_HIP, mdg.MDG_ERR_DEVICE)
    assert mdg.mdg_dgemm_crt("N", "N", 64, 64, 64, 1.0, fake, 63, fake, 64, 0.0, fake, 64, 0,
                             fake, 0) == 8   # an earlier bad argument is reported first
    assert mdg.mdg_crt_residues(0, "N", 64, 64, fake, 64, 15, 73, fake, fake) == 8

"""The 2-D tensor form of the binding (gemm2d_args) on the CPU: the dgemm call it derives from
shapes and strides, run through the oracle on the same storage, computes alpha op(A) op(B) + beta C
for every mix of column-major and row-major operands, transpose flags and padded leading
dimensions (integer data: exact)."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from paper_1609_00076_amd.binding import gemm2d_args


def _stored(x, layout, pad):
    """(flat storage, 2-D view with x's values, element strides) in the given layout."""
    r, c = x.shape
    if layout == "col":
        ld = r + pad
        flat = np.full(ld * c, np.nan)
        view = flat.reshape(c, ld)[:, :r].T
    else:
        ld = c + pad
        flat = np.full(ld * r, np.nan)
        view = flat.reshape(r, ld)[:, :c]
    view[:, :] = x
    return flat, view, tuple(s // 8 for s in view.strides)


@pytest.mark.parametrize("la,lb,lc", list(itertools.product(["col", "row"], repeat=3)))
@pytest.mark.parametrize("trans", ["NN", "NT", "TN", "TT"])
def test_every_layout_mix_matches_the_definition(la, lb, lc, trans):
    g = synth.rng(synth.seed_for(30, 0, 0))
    m, n, k = 7, 5, 6
    opa = g.integers(-8, 9, (m, k)).astype(np.float64)
    opb = g.integers(-8, 9, (k, n)).astype(np.float64)
    c0 = g.integers(-8, 9, (m, n)).astype(np.float64)
    a = opa.T if trans[0] == "T" else opa
    b = opb.T if trans[1] == "T" else opb
    fa, va, sa = _stored(a, la, 2)
    fb, vb, sb = _stored(b, lb, 1)
    fc, vc, sc = _stored(c0, lc, 3)
    ta, tb, mm, nn, kk, lda, ldb, ldc, swap = gemm2d_args(a.shape, sa, b.shape, sb, c0.shape, sc,
                                                        trans[0], trans[1])
    first, second = (fb, fa) if swap else (fa, fb)
    assert oracle.dgemm(ta, tb, mm, nn, kk, 1.5, first, lda, second, ldb, -0.5, fc, ldc) == 0
    assert np.array_equal(vc, 1.5 * opa @ opb - 0.5 * c0)


def test_unit_dimensions_and_refusals():
    # a column (m x 1) and a row (1 x k) are both layouts whatever the other stride
    assert gemm2d_args((4, 1), (1, 1), (1, 3), (3, 1), (4, 3), (1, 4))[:8] == \
        ("N", "N", 4, 3, 1, 4, 1, 4)
    with pytest.raises(ValueError):   # neither stride is 1
        gemm2d_args((4, 4), (8, 2), (4, 4), (1, 4), (4, 4), (1, 4))
    with pytest.raises(ValueError):   # column-major with ld < rows
        gemm2d_args((4, 4), (1, 3), (4, 4), (1, 4), (4, 4), (1, 4))
    with pytest.raises(ValueError):   # shapes that do not chain
        gemm2d_args((4, 3), (1, 4), (4, 4), (1, 4), (4, 4), (1, 4))

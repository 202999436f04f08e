"""Pins for the oracle's entry groupings (CPU only)."""
import numpy as np
import pytest

from oracle import mach as O
from oracle import segments as S


@pytest.mark.parametrize("shape,h,perm", [((4, 3, 5), 2, [1, 0]), ((4, 3, 5), 2, [0, 1]),
                                          ((3, 2, 4, 5), 2, [0, 1]), ((6, 7), 1, [0]),
                                          ((5, 4, 3), 1, [0])])
def test_column_order_matches_loops(shape, h, perm):
    X = np.random.default_rng(0).standard_normal(shape)
    coo = O.sample_coo(X, 0.4, 3, 1)
    o1, c1 = S.column_order(coo.idx, shape, h, perm)
    o2, c2 = S.column_order_loops(coo.idx, shape, h, perm)
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_array_equal(c1, c2)


def test_row_pointers_by_hand():
    shape = (2, 3, 4)                      # h = 1: rows i0, 12 columns each
    idx = np.array([0, 5, 11, 12, 13, 23], dtype=np.uint32)
    np.testing.assert_array_equal(S.row_pointers(idx, shape, 1), [0, 3, 6])
    np.testing.assert_array_equal(S.row_pointers(idx, shape, 2), [0, 1, 2, 3, 5, 5, 6])


@pytest.mark.parametrize("shape", [(4, 3, 5), (6, 7), (3, 2, 4, 5), (5, 4, 3)])
def test_groups_are_rows_of_the_matricization(shape):
    """With one head mode the row groups hold exactly the kept entries of
    each row of the mode-0 matricization (Section 2.1); with one tail mode
    the column groups hold those of each row of the last mode's."""
    X = np.random.default_rng(1).standard_normal(shape)
    coo = O.sample_coo(X, 0.5, 5, 2)
    Xk = O.dense_from_coo(coo, scale_by_p=False)
    d = len(shape)
    ptr = S.row_pointers(coo.idx, shape, 1)
    U0 = O.unfold(Xk, 0)
    for r in range(shape[0]):
        got = sorted(coo.val[ptr[r]:ptr[r + 1]].astype(np.float64).tolist())
        want = sorted(U0[r][np.flatnonzero(U0[r])].tolist())
        assert got == want
    order, colptr = S.column_order(coo.idx, shape, d - 1, list(range(d - 1)))
    Ul = O.unfold(Xk, d - 1)
    vals = coo.val[order].astype(np.float64)
    for c in range(shape[-1]):
        got = sorted(vals[colptr[c]:colptr[c + 1]].tolist())
        want = sorted(Ul[c][np.flatnonzero(Ul[c])].tolist())
        assert got == want


def test_head_split_by_hand():
    assert S.head_split((128, 16, 16384)) == (2, [1, 0])      # 2048 rows x 16384 columns
    assert S.head_split((64, 32, 48)) == (1, [0])             # 64 x 1536 beats 2048 x 48
    assert S.head_split((300, 200)) == (1, [0])
    assert S.head_split((64, 64, 64, 256)) == (2, [0, 1])     # 4096 x 16384; equal dims by mode
    assert S.head_split((2, 3, 4, 5, 6)) == (2, [0, 1])       # d = 5: h = d // 2

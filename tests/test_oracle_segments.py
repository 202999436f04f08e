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

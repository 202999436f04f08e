"""Plain definitions of the groupings of the kept entries (oracle side).

TEST INFRASTRUCTURE ONLY.

The kept entries of X-hat are grouped as rows of a matricization before
any mode product is taken: the matricization of Section 2.1 puts element
(i_1..i_d) in row i_k.  The GPU path groups them in two ways, for a split of
the modes into head modes 0..h-1 and tail modes h..d-1:
  * by head row r (C-order index over the head modes): the entries in
    ascending linear-index order, with row pointers;
  * by tail column c (C-order index over the tail modes): within a column,
    ordered by the head coordinates taken in a given order (outermost
    first), with column pointers.
Both are written here as sorts and counts (numpy lexsort / bincount), which
is their definition.  `head_split` states which split and head order the
library declares for a shape (mach_layout_info), so that a test takes them
from this stated rule and never from the library.  Pinned by
tests/test_oracle_segments.py against brute-force Python loops, against the
rows of Section 2.1's matricization, and (host side only) against the
library's declared split.
"""
from __future__ import annotations

import numpy as np


def head_split(shape):
    """The split of the modes into head modes 0..h-1 and tail modes h..d-1
    and the order of the head coordinates inside a tail column, by the rule
    the library states: h ranges over [max(1, d-2), min(2, d-1)] (d//2 when
    that range is empty), and the h whose head rows and tail columns are the
    most balanced (smallest |log2 MH - log2 MT|, the first on ties) is taken;
    head coordinates are ordered by ascending (dimension, mode), outermost
    first, so the largest head mode varies fastest."""
    dims = [int(x) for x in shape]
    d = len(dims)
    N = float(np.prod(dims))
    lo, hi = max(1, d - 2), min(2, d - 1)
    if lo > hi:
        lo = hi = d // 2
    best, bestv = lo, None
    for h in range(lo, hi + 1):
        mh = float(np.prod(dims[:h]))
        v = abs(np.log2(mh) - np.log2(N / mh))
        if bestv is None or v < bestv - 1e-12:
            best, bestv = h, v
    perm = sorted(range(best), key=lambda m: (dims[m], m))
    return best, perm


def row_pointers(idx: np.ndarray, shape, h: int) -> np.ndarray:
    """Row pointers of the head-row grouping (entries already in l order)."""
    MT = int(np.prod(shape[h:]))
    MH = int(np.prod(shape[:h]))
    r = idx.astype(np.int64) // MT
    return np.concatenate([[0], np.cumsum(np.bincount(r, minlength=MH))]).astype(np.int64)


def column_order(idx: np.ndarray, shape, h: int, headperm):
    """Permutation of the entries into the tail-column grouping, and the
    column pointers.  Within a column, entries are sorted by the head
    coordinates in headperm order (headperm[0] outermost)."""
    shape = tuple(int(s) for s in shape)
    MT = int(np.prod(shape[h:]))
    lin = idx.astype(np.int64)
    coords = np.unravel_index(lin, shape)
    c = lin % MT
    keys = [coords[m] for m in reversed(list(headperm))] + [c]
    order = np.lexsort(keys)
    colptr = np.concatenate([[0], np.cumsum(np.bincount(c, minlength=MT))]).astype(np.int64)
    return order, colptr


def column_order_loops(idx, shape, h, headperm):
    """The same grouping by explicit loops over columns and head positions
    (tiny tensors only)."""
    shape = tuple(int(s) for s in shape)
    MT = int(np.prod(shape[h:]))
    kept = set(int(x) for x in idx)
    pos = {int(x): k for k, x in enumerate(idx)}
    head_dims = [shape[m] for m in headperm]
    order = []
    colptr = [0]
    for c in range(MT):
        for t in np.ndindex(*head_dims):
            hc = [0] * h
            for j, m in enumerate(headperm):
                hc[m] = t[j]
            r = 0
            for m in range(h):
                r = r * shape[m] + hc[m]
            lin = r * MT + c
            if lin in kept:
                order.append(pos[lin])
        colptr.append(len(order))
    return np.array(order, dtype=np.int64), np.array(colptr, dtype=np.int64)

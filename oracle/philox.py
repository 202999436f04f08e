"""Philox counter-based generator, written from its published definition.

Test infrastructure only (see oracle/__init__.py): nothing in the product
path may import this module.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, Section 3.3 (the Philox
S-box: two multiplications, a hi/lo split and an xor with the round key)
and Section 3.3's constants table.

The paper being implemented (MACH) keeps each entry with probability p by
an independent coin toss (Alg. 1 and Alg. 2, the MACH comment block;
Remark 1) and names no generator.  The reading taken here is one
independent Bernoulli(p) draw per linear index, produced by Philox4x32-10
keyed by (seed, window); see `mask_words` for the counter layout.

Two implementations live here:
  * `philox_block`  - one block, Python integers, any word width (32 or 64).
                      Slow and obviously a transcription of the definition.
  * `philox4x32_10` - numpy uint64 arithmetic over arrays of counters.  The
                      products of two uint32 values are exact in uint64.
The tests pin `philox_block` against published known-answer vectors (W=32)
and against numpy's own Philox4x64-10 bit generator (W=64), and pin the
vectorised form against `philox_block`.
"""
from __future__ import annotations

import numpy as np

# Multipliers and Weyl key increments (SC'11, Philox constants).
_CONST = {
    32: dict(M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85),
    64: dict(M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
             W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B),
}


def philox_block(ctr, key, width=32, rounds=10):
    """One Philox4xW block.  ctr: 4 words, key: 2 words (Python ints).

    Round r (r = 0..rounds-1) uses the key bumped r times by (W0, W1).
    A round maps (c0, c1, c2, c3) to
        (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)).
    """
    c = _CONST[width]
    mask = (1 << width) - 1
    c0, c1, c2, c3 = (int(x) & mask for x in ctr)
    k0, k1 = (int(x) & mask for x in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + c["W0"]) & mask
            k1 = (k1 + c["W1"]) & mask
        p0 = c["M0"] * c0
        p1 = c["M1"] * c2
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments are uint32 arrays (or scalars)
    that broadcast together.  Returns four uint32 arrays."""
    c = _CONST[32]
    m32 = np.uint64(0xFFFFFFFF)
    sh = np.uint64(32)
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64)
    k1 = np.asarray(k1, dtype=np.uint64)
    M0, M1 = np.uint64(c["M0"]), np.uint64(c["M1"])
    W0, W1 = np.uint64(c["W0"]), np.uint64(c["W1"])
    for r in range(10):
        if r:
            k0 = (k0 + W0) & m32
            k1 = (k1 + W1) & m32
        p0 = M0 * c0          # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> sh, p0 & m32
        hi1, lo1 = p1 >> sh, p1 & m32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def mask_words(lin, seed, window_id):
    """The 32-bit random word attached to each linear index `lin` (uint64 array).

    Counter layout (the reading taken here; the paper fixes none):
        counter = (q mod 2^32, q >> 32, window mod 2^32, window >> 32), q = lin // 4
        key     = (seed mod 2^32, seed >> 32)
        word    = output word number (lin mod 4) of that block.
    """
    lin = np.asarray(lin, dtype=np.uint64)
    q = lin >> np.uint64(2)
    w = np.uint64(window_id)
    s = np.uint64(seed)
    m32 = np.uint64(0xFFFFFFFF)
    outs = philox4x32_10(q & m32, q >> np.uint64(32), w & m32, w >> np.uint64(32),
                         s & m32, s >> np.uint64(32))
    sel = (lin & np.uint64(3)).astype(np.int64)
    stacked = np.stack(outs, axis=0)
    return np.take_along_axis(stacked, sel[None, ...], axis=0)[0]


def mask_words_ticks(series, tick, seed):
    """The 32-bit word of a measurement of series `series` at absolute tick
    `tick` (uint64 arrays that broadcast together) under tick-keyed coins.

    Counter layout (the reading taken here for streams, Remark 2):
        counter = (q mod 2^32, q >> 32, series, 0), q = tick // 4
        key     = (seed mod 2^32, seed >> 32)
        word    = output word number (tick mod 4) of that block.
    """
    series = np.asarray(series, dtype=np.uint64)
    tick = np.asarray(tick, dtype=np.uint64)
    series, tick = np.broadcast_arrays(series, tick)
    q = tick >> np.uint64(2)
    s = np.uint64(seed)
    m32 = np.uint64(0xFFFFFFFF)
    outs = philox4x32_10(q & m32, q >> np.uint64(32), series & m32, np.zeros_like(q),
                         s & m32, s >> np.uint64(32))
    sel = (tick & np.uint64(3)).astype(np.int64)
    stacked = np.stack(outs, axis=0)
    return np.take_along_axis(stacked, sel[None, ...], axis=0)[0]

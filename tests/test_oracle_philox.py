"""Pins for the oracle's Philox generator (CPU only)."""
import os

import numpy as np
import pytest

from oracle import philox


def _kat_rows(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(x, 16) for x in line.split()]
            rows.append((vals[:4], vals[4:6], tuple(vals[6:10])))
    return rows


def test_philox4x32_known_answers(golden_dir):
    rows = _kat_rows(golden_dir)
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert philox.philox_block(ctr, key, 32, 10) == want


@pytest.mark.parametrize("counter,key", [(0, 0), (12345, 678), (2**64 - 2, 2**127 + 5),
                                         (2**200 % 2**256 + 99, 31337)])
def test_philox4x64_matches_numpy_bit_generator(counter, key):
    """numpy's Philox (4x64-10) shares the round structure: an independent
    library implementation of the same definition.  numpy bumps the
    256-bit counter before producing each block."""
    bg = np.random.Philox(counter=counter, key=key)
    got = tuple(int(x) for x in bg.random_raw(4))
    c = (counter + 1) % (1 << 256)
    ctr = [(c >> (64 * i)) & (2**64 - 1) for i in range(4)]
    k = [(key >> (64 * i)) & (2**64 - 1) for i in range(2)]
    assert philox.philox_block(ctr, k, 64, 10) == got


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(4, 300), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(2, 300), dtype=np.uint64)
    out = philox.philox4x32_10(*ctr, *key)
    for j in range(300):
        want = philox.philox_block([int(c[j]) for c in ctr], [int(k[j]) for k in key], 32, 10)
        assert tuple(int(o[j]) for o in out) == want


def test_mask_word_layout():
    """word(l) = output number (l mod 4) of the block with counter
    (q lo, q hi, window lo, window hi), q = l // 4, key = (seed lo, seed hi)."""
    seed, win = 0x1234_5678_9ABC_DEF0, 0x0F0E_0D0C_0B0A_0908
    lins = np.array([0, 1, 2, 3, 4, 7, 1 << 33, (1 << 40) + 3], dtype=np.uint64)
    words = philox.mask_words(lins, seed, win)
    for l, w in zip(lins.tolist(), words.tolist()):
        q = l // 4
        blk = philox.philox_block([q & 0xFFFFFFFF, q >> 32, win & 0xFFFFFFFF, win >> 32],
                                  [seed & 0xFFFFFFFF, seed >> 32], 32, 10)
        assert w == blk[l % 4]


def test_planted_round_mistake_is_caught(golden_dir, monkeypatch):
    """A plausible transcription error (the two xor partners swapped) must
    fail the known-answer pin."""
    real = philox.philox_block

    def wrong(ctr, key, width=32, rounds=10):
        c = philox._CONST[width]
        mask = (1 << width) - 1
        c0, c1, c2, c3 = ctr
        k0, k1 = key
        for r in range(rounds):
            if r:
                k0 = (k0 + c["W0"]) & mask
                k1 = (k1 + c["W1"]) & mask
            p0, p1 = c["M0"] * c0, c["M1"] * c2
            c0, c1, c2, c3 = (p1 >> width) ^ c3 ^ k0, p1 & mask, (p0 >> width) ^ c1 ^ k1, p0 & mask
        return (c0, c1, c2, c3)

    monkeypatch.setattr(philox, "philox_block", wrong)
    bad = [philox.philox_block(ctr, key) == want for ctr, key, want in _kat_rows(golden_dir)]
    assert not all(bad)
    monkeypatch.setattr(philox, "philox_block", real)

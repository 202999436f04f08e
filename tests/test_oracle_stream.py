"""Pins of the oracle's tick-keyed coins for stream windows (reading R9):
the vectorised mask against one Philox block per entry from its published
definition, the overlap property, and the 64-bit tick counter."""
import numpy as np

from oracle import mach as O
from oracle.philox import philox_block


def _brute(shape, p, seed, tick0):
    T = shape[-1]
    nser = int(np.prod(shape[:-1]))
    thr = O.keep_threshold(p)
    out = np.zeros((nser, T), dtype=bool)
    for j in range(nser):
        for t in range(T):
            tau = tick0 + t
            q = tau // 4
            words = philox_block((q & 0xFFFFFFFF, q >> 32, j, 0), (seed & 0xFFFFFFFF, seed >> 32))
            out[j, t] = words[tau % 4] < thr
    return out.reshape(shape)


def test_mask_matches_one_block_per_entry():
    for shape, p, seed, tick0 in [((2, 3, 9), 0.4, 0x1234567890, 6),
                                  ((5, 7), 0.5, 3, 2**33 + 1),     # tick/4 has a high word
                                  ((2, 2, 2, 13), 0.3, 2**63 + 5, 3)]:
        np.testing.assert_array_equal(O.sample_mask_ticks(shape, p, seed, tick0),
                                      _brute(shape, p, seed, tick0))


def test_overlapping_windows_share_their_coins():
    seed, p = 77, 0.3
    a = O.sample_mask_ticks((3, 2, 40), p, seed, 5)       # ticks 5 .. 44
    b = O.sample_mask_ticks((3, 2, 40), p, seed, 17)      # ticks 17 .. 56
    np.testing.assert_array_equal(a[..., 12:], b[..., :28])
    # a different seed, or the window-keyed coin, gives other coins
    assert not np.array_equal(a, O.sample_mask_ticks((3, 2, 40), p, seed + 1, 5))
    assert not np.array_equal(a, O.sample_mask((3, 2, 40), p, seed, 5))


def test_keep_rate_and_series_independence():
    m = O.sample_mask_ticks((64, 4096), 0.1, 5, 1000)
    assert abs(m.mean() - 0.1) < 5 * np.sqrt(0.1 * 0.9 / m.size)
    # different series see different coins at the same ticks
    assert np.mean(m[0] == m[1]) < 0.9


def test_mask_words_ticks_against_one_block_per_word():
    from oracle.philox import mask_words_ticks
    seed = 0xDEADBEEF12345
    series = np.array([0, 1, 7, 2**31 + 3], dtype=np.uint64)[:, None]
    ticks = np.array([0, 1, 2, 3, 4, 5, 2**32 * 4 + 2, 2**40 + 7], dtype=np.uint64)[None, :]
    got = mask_words_ticks(series, ticks, seed)
    for a, j in enumerate(series[:, 0]):
        for b, tau in enumerate(ticks[0]):
            j, tau = int(j), int(tau)
            q = tau // 4
            w = philox_block((q & 0xFFFFFFFF, q >> 32, j, 0), (seed & 0xFFFFFFFF, seed >> 32))
            assert int(got[a, b]) == w[tau % 4], (j, tau)


def test_coo_and_dense_of_a_stream_window():
    """The COO list and dense X-hat of a tick-keyed window follow its mask,
    and two overlapping windows of one stream agree on the shared ticks."""
    rng = np.random.default_rng(4)
    Xl = rng.standard_normal((3, 2, 60)).astype(np.float32)
    p, seed = 0.3, 99
    a, b = Xl[..., 0:40], Xl[..., 25:60]                   # ticks 100..139 and 125..159
    mask = _brute(a.shape, p, seed, 100)
    coo = O.sample_coo_ticks(np.ascontiguousarray(a), p, seed, 100)
    np.testing.assert_array_equal(coo.idx, np.flatnonzero(mask.ravel()))
    np.testing.assert_array_equal(coo.val, a.ravel()[coo.idx])
    assert coo.sumsq == float(np.sum(a.ravel()[coo.idx].astype(np.float64) ** 2))
    Xa = O.sampled_tensor_ticks(np.ascontiguousarray(a), p, seed, 100)
    np.testing.assert_array_equal(Xa, np.where(mask, a.astype(np.float64) / p, 0.0))
    Xb = O.sampled_tensor_ticks(np.ascontiguousarray(b), p, seed, 125)
    np.testing.assert_array_equal(Xa[..., 25:40], Xb[..., 0:15])

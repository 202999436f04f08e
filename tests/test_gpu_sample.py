"""GPU parity of the coin toss and the sparse layouts (bit-exact)."""
import math

import numpy as np
import pytest

import synth
from oracle import mach as O
from oracle import segments as S
from tests.gpu_helpers import pack_mask, say

pytestmark = pytest.mark.gpu

CASES = [
    ("tucker-64x32x48-f64", (64, 32, 48), "f64", 0.1, 20261, 0),
    ("monitor-32x16x1000", (32, 16, 1000), "f32", 0.1, 7, 3),
    ("voxel-16x16x16x32", (16, 16, 16, 32), "f32", 0.05, 11, 1),
    ("matrix-37x53", (37, 53), "f32", 0.3, 5, 2),
    ("all-kept-5x7x9", (5, 7, 9), "f32", 1.0, 1, 0),
    ("p0.01-128x16x2048", (128, 16, 2048), "f32", 0.01, 3, 9),
    ("ragged-3x5x7x11", (3, 5, 7, 11), "f64", 0.5, 99, 2**40 + 3),
]


def _input(shape, dt, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(shape)
    return X.astype(np.float64 if dt == "f64" else np.float32)


@pytest.mark.parametrize("name,shape,dt,p,seed,win", CASES, ids=[c[0] for c in CASES])
def test_sample_and_layouts_bit_exact(name, shape, dt, p, seed, win):
    import torch
    from paper_0909_4969_amd import mach as M
    X = _input(shape, dt, seed)
    coo = O.sample_coo(X, p, seed, win)
    say("sample", name, shape, p)
    sw = M.sample(torch.from_numpy(X).cuda(), p, seed, win)
    st, nnz, ss = sw.status()
    assert st == 0
    assert nnz == coo.nnz
    idx, val = sw.entries("coo_l", nnz)
    np.testing.assert_array_equal(idx, coo.idx)
    np.testing.assert_array_equal(val.view(np.uint32), coo.val.view(np.uint32))
    assert abs(ss - coo.sumsq) <= 1e-12 * max(coo.sumsq, 1e-300)
    N = int(np.prod(shape))
    nwords = ((N + 16383) // 16384) * 256
    mask = O.sample_mask(shape, p, seed, win).ravel()
    words = sw.u64("bitmap", nwords)
    np.testing.assert_array_equal(words, pack_mask(mask, nwords))
    pc = np.array([bin(int(w)).count("1") for w in words], dtype=np.int64)
    wr = sw.u32("wrank", nwords + 1).astype(np.int64)
    np.testing.assert_array_equal(wr, np.concatenate([[0], np.cumsum(pc)]))
    h, perm = M.layout_info(shape)
    MH = int(np.prod(shape[:h]))
    MT = N // MH
    np.testing.assert_array_equal(sw.u32("rowptr", MH + 1), S.row_pointers(coo.idx, shape, h))
    order, colptr = S.column_order(coo.idx, shape, h, perm)
    np.testing.assert_array_equal(sw.u32("colptr", MT + 1), colptr)
    tidx, tval = sw.entries("coo_t", nnz)
    np.testing.assert_array_equal(tidx, coo.idx[order])
    np.testing.assert_array_equal(tval.view(np.uint32), coo.val[order].view(np.uint32))


def test_capacity_overflow_sets_status():
    import torch
    from paper_0909_4969_amd import mach as M
    X = _input((16, 16, 64), "f32", 1)
    say("sample overflow")
    sw = M.sample(torch.from_numpy(X).cuda(), 0.5, 1, 0, cap=100)
    st, nnz, _ = sw.status()
    assert st == M.MACH_ENOMEM
    assert nnz == O.sample_coo(X, 0.5, 1, 0).nnz


def test_invalid_arguments_rejected_on_host():
    import torch
    from paper_0909_4969_amd import mach as M
    X = torch.zeros(4, 5, 6, device="cuda")
    for p in (0.0, -1.0, 1.5, float("nan")):
        with pytest.raises(M.MachError):
            M.sample(X, p, 0, 0, cap=100)
    with pytest.raises(M.MachError):
        M.sample(X, 0.5, 0, 0, cap=0)


def test_full_size_monitoring_tensor_sampled_positions():
    """128x16x16384 at p = 0.1 (the benchmarked workload): the kept count is
    Binomial, and the mask, the kept entries and the column copy agree with
    the oracle on sampled windows of the linear index."""
    import torch
    from paper_0909_4969_amd import mach as M
    shape, p, seed, win = (128, 16, 16384), 0.1, 20262, 0
    X, _ = synth.workload2(shape)
    say("sample full-size", shape)
    sw = M.sample(torch.from_numpy(X).cuda(), p, seed, win)
    st, nnz, ss = sw.status()
    assert st == 0
    N = X.size
    q = O.keep_threshold(p) / 2**32
    assert abs(nnz - N * q) < 6 * math.sqrt(N * q * (1 - q))
    idx, val = sw.entries("coo_l", nnz)
    assert np.all(np.diff(idx.astype(np.int64)) > 0)
    rng = np.random.default_rng(1)
    flat = X.ravel()
    for start in rng.integers(0, N - 70000, 8):
        lo, hi = int(start), int(start) + 65536
        lin = np.arange(lo, hi, dtype=np.uint64)
        keep = O.mask_words(lin, seed, win).astype(np.uint64) < np.uint64(O.keep_threshold(p))
        want = np.flatnonzero(keep).astype(np.int64) + lo
        sel = (idx >= lo) & (idx < hi)
        np.testing.assert_array_equal(idx[sel].astype(np.int64), want)
        np.testing.assert_array_equal(val[sel], flat[want])
    assert abs(ss - float(np.sum(flat[idx].astype(np.float64) ** 2))) <= 1e-10 * ss
    h, perm = M.layout_info(shape)
    order, colptr = S.column_order(idx, shape, h, perm)
    MT = N // int(np.prod(shape[:h]))
    np.testing.assert_array_equal(sw.u32("colptr", MT + 1), colptr)
    tidx, _ = sw.entries("coo_t", nnz)
    np.testing.assert_array_equal(tidx, idx[order])

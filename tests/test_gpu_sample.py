"""GPU parity of the coin toss and the sparse layouts (bit-exact)."""
import math

import numpy as np
import pytest

import synth
from oracle import mach as O
from oracle import segments as S
from tests.gpu_helpers import columns_elementwise, pack_mask, say, sin_theta, subspace_tol

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
    h, perm = S.head_split(shape)
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


FULL = [("monitoring-128x16x16384-p0.1", 0.1, 20262), ("monitoring-128x16x16384-p0.01", 0.01, 20262),
        ("voxel-64x64x64x256-p0.05", 0.05, 20263)]


@pytest.mark.parametrize("name,p,seed", FULL, ids=[c[0] for c in FULL])
def test_full_size_whole_mask(name, p, seed):
    """The full-size workloads (the monitoring window at p = 0.1 and 0.01,
    the 4-way voxel tensor at p = 0.05): the whole keep bitmap (every coin),
    the kept entries, their sum of squares and both layouts agree with the
    oracle bit for bit."""
    import torch
    from paper_0909_4969_amd import mach as M
    win = 0
    X, _ = synth.workload3() if name.startswith("voxel") else synth.workload2()
    shape = X.shape
    say("sample full-size", name, shape)
    sw = M.sample(torch.from_numpy(X).cuda(), p, seed, win)
    st, nnz, ss = sw.status()
    assert st == 0
    N = X.size
    coo = O.sample_coo(X, p, seed, win)
    assert nnz == coo.nnz
    nwords = ((N + 16383) // 16384) * 256
    words = sw.u64("bitmap", nwords)
    np.testing.assert_array_equal(words, pack_mask(O.sample_mask(shape, p, seed, win).ravel(), nwords))
    idx, val = sw.entries("coo_l", nnz)
    np.testing.assert_array_equal(idx, coo.idx)
    np.testing.assert_array_equal(val.view(np.uint32), coo.val.view(np.uint32))
    assert abs(ss - coo.sumsq) <= 1e-12 * coo.sumsq
    h, perm = S.head_split(shape)
    MH = int(np.prod(shape[:h]))
    np.testing.assert_array_equal(sw.u32("rowptr", MH + 1), S.row_pointers(coo.idx, shape, h))
    order, colptr = S.column_order(coo.idx, shape, h, perm)
    np.testing.assert_array_equal(sw.u32("colptr", N // MH + 1), colptr)
    tidx, tval = sw.entries("coo_t", nnz)
    np.testing.assert_array_equal(tidx, coo.idx[order])
    np.testing.assert_array_equal(tval.view(np.uint32), coo.val[order].view(np.uint32))


TICK_CASES = [
    ("ticks-128x16x2048", (128, 16, 2048), "f32", 0.1, 5, 1000003),      # T a multiple of 64
    ("ticks-7x5x333", (7, 5, 333), "f32", 0.3, 6, 2**32 + 1),            # ragged T, high tick word
    ("ticks-64x100", (64, 100), "f64", 0.5, 7, 0),
    ("ticks-4x4x4x97", (4, 4, 4, 97), "f32", 0.2, 2**63 + 9, 2),
]


@pytest.mark.parametrize("name,shape,dt,p,seed,tick0", TICK_CASES, ids=[c[0] for c in TICK_CASES])
def test_tick_keyed_sample_bit_exact(name, shape, dt, p, seed, tick0):
    """mach_sample_ticks against the oracle's tick-keyed coins (reading R9):
    bitmap, COO and the layouts built from them, bit for bit."""
    import torch
    from paper_0909_4969_amd import mach as M
    X = _input(shape, dt, seed % 1000)
    coo = O.sample_coo_ticks(X, p, seed, tick0)
    say("sample ticks", name, shape, p, tick0)
    sw = M.sample(torch.from_numpy(X).cuda(), p, seed, 0, tick0=tick0)
    st, nnz, ss = sw.status()
    assert st == 0
    assert nnz == coo.nnz
    idx, val = sw.entries("coo_l", nnz)
    np.testing.assert_array_equal(idx, coo.idx)
    np.testing.assert_array_equal(val.view(np.uint32), coo.val.view(np.uint32))
    assert abs(ss - coo.sumsq) <= 1e-12 * max(coo.sumsq, 1e-300)
    N = int(np.prod(shape))
    nwords = ((N + 16383) // 16384) * 256
    words = sw.u64("bitmap", nwords)
    np.testing.assert_array_equal(words, pack_mask(O.sample_mask_ticks(shape, p, seed, tick0).ravel(), nwords))
    h, perm = S.head_split(shape)
    MH = int(np.prod(shape[:h]))
    np.testing.assert_array_equal(sw.u32("rowptr", MH + 1), S.row_pointers(coo.idx, shape, h))


def test_overlapping_stream_windows_keep_the_same_measurements():
    """Two windows of one stream that overlap in time keep exactly the same
    measurements (and values) in the overlap."""
    import torch
    from paper_0909_4969_amd import mach as M
    rng = np.random.default_rng(8)
    series = rng.standard_normal((16, 8, 1800)).astype(np.float32)   # ticks 500 .. 2299
    T, t0a, t0b, p, seed = 1024, 500, 884, 0.1, 42
    kept = []
    for t0 in (t0a, t0b):
        Xw = np.ascontiguousarray(series[..., t0 - 500:t0 - 500 + T])
        say("sample window ticks", t0)
        sw = M.sample(torch.from_numpy(Xw).cuda(), p, seed, 0, tick0=t0)
        st, nnz, _ = sw.status()
        assert st == 0
        idx, val = sw.entries("coo_l", nnz)
        j, t = idx.astype(np.int64) // T, idx.astype(np.int64) % T
        kept.append({(int(a), int(b) + t0): v for a, b, v in zip(j, t, val.view(np.uint32))})
    lo, hi = t0b, t0a + T
    ov = [{k: v for k, v in d.items() if lo <= k[1] < hi} for d in kept]
    assert len(ov[0]) > 1000
    assert ov[0] == ov[1]


def _workspace_arrays(sw, shape, nnz):
    """Everything the layouts hold, as host arrays, for bit-for-bit
    comparison of two sample workspaces of the same shape and capacity."""
    N = int(np.prod(shape))
    nwords = ((N + 16383) // 16384) * 256
    h, _ = S.head_split(shape)
    MH = int(np.prod(shape[:h]))
    MT = N // MH
    out = {"bitmap": sw.u64("bitmap", nwords), "wrank": sw.u32("wrank", nwords + 1),
           "rowptr": sw.u32("rowptr", MH + 1), "colptr": sw.u32("colptr", MT + 1)}
    for which in ("coo_l", "coo_t"):
        idx, val = sw.entries(which, nnz)
        out[which + "_idx"], out[which + "_val"] = idx, val.view(np.uint32)
    return out


# (name, stream shape (series..., ticks), window T, first ticks of the
# earlier and the new window, dtype, p, seed of the earlier window)
SLIDES = [
    ("forward-7x5x333", (7, 5), 333, (1000, 1100), np.float32, 0.3, 61),
    ("forward-hop1-32x16x2048", (32, 16), 2048, (5000, 5001), np.float32, 0.1, 62),
    ("backward-16x8x600", (16, 8), 600, (3000, 2700), np.float32, 0.2, 63),
    ("no-overlap-16x8x600", (16, 8), 600, (0, 600), np.float32, 0.2, 64),
    ("other-seed-16x8x600", (16, 8), 600, (0, 150), np.float32, 0.2, None),
    ("f64-9x64x500", (9, 64), 500, (10, 210), np.float64, 0.25, 65),
]


@pytest.mark.parametrize("name,series,T,ticks,dt,p,seed0", SLIDES, ids=[x[0] for x in SLIDES])
def test_slid_window_equals_fresh_toss(name, series, T, ticks, dt, p, seed0):
    """mach_sample_ticks_slide from an earlier window's sample against a fresh
    mach_sample_ticks of the new window: every array of the workspace bit for
    bit, the kept count and the sum of squares; and the mask and kept list
    against the oracle's tick-keyed coins.  "other-seed" gives the earlier
    window another seed, so nothing may be reused (fresh toss)."""
    import torch
    from paper_0909_4969_amd import mach as M
    seed = 66
    t_prev, t_new = ticks
    lo = min(t_prev, t_new)
    rng = np.random.default_rng(sum(map(ord, name)))
    stream = rng.standard_normal(tuple(series) + (max(t_prev, t_new) + T - lo,)).astype(dt)
    X_prev = np.ascontiguousarray(stream[..., t_prev - lo:t_prev - lo + T])
    X_new = np.ascontiguousarray(stream[..., t_new - lo:t_new - lo + T])
    shape = X_new.shape
    cap = M.nnz_capacity(shape, p)
    say("slide", name, shape, ticks, p)
    prev = M.sample(torch.from_numpy(X_prev).cuda(), p, seed if seed0 is not None else seed + 1, 0,
                    cap=cap, tick0=t_prev)
    Xd = torch.from_numpy(X_new).cuda()
    slid = M.sample(Xd, p, seed, 0, cap=cap, tick0=t_new, prev=prev)
    fresh = M.sample(Xd, p, seed, 0, cap=cap, tick0=t_new)
    st_s, nnz_s, ss_s = slid.status()
    st_f, nnz_f, ss_f = fresh.status()
    assert st_s == 0 and st_f == 0
    assert nnz_s == nnz_f and ss_s == ss_f
    a, b = _workspace_arrays(slid, shape, nnz_s), _workspace_arrays(fresh, shape, nnz_f)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    coo = O.sample_coo_ticks(X_new, p, seed, t_new)
    assert nnz_s == coo.nnz
    np.testing.assert_array_equal(a["coo_l_idx"], coo.idx)
    np.testing.assert_array_equal(a["coo_l_val"], coo.val.view(np.uint32))


def test_slid_monitoring_window():
    """A 128 x 16 x 16384 window slid by 2048 ticks along its stream: bit for
    bit a fresh toss (float32 input, p = 0.1)."""
    import torch
    from paper_0909_4969_amd import mach as M
    rng = np.random.default_rng(71)
    T, hop, p, seed = 16384, 2048, 0.1, 72
    stream = torch.from_numpy(rng.standard_normal((128, 16, T + hop)).astype(np.float32)).cuda()
    Xa = stream[..., :T].contiguous()
    Xb = stream[..., hop:].contiguous()
    cap = M.nnz_capacity((128, 16, T), p)
    say("slide monitoring window", hop)
    prev = M.sample(Xa, p, seed, 0, cap=cap, tick0=40000)
    slid = M.sample(Xb, p, seed, 0, cap=cap, tick0=40000 + hop, prev=prev)
    fresh = M.sample(Xb, p, seed, 0, cap=cap, tick0=40000 + hop)
    st_s, nnz_s, ss_s = slid.status()
    st_f, nnz_f, ss_f = fresh.status()
    assert st_s == 0 and st_f == 0 and nnz_s == nnz_f and ss_s == ss_f
    a, b = _workspace_arrays(slid, (128, 16, T), nnz_s), _workspace_arrays(fresh, (128, 16, T), nnz_f)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_tick_keyed_window_through_hosvd():
    """The solver on a tick-keyed sample matches the oracle's HOSVD of the
    same sampled tensor."""
    import torch
    from paper_0909_4969_amd import mach as M
    X, _ = synth.workload2(shape=(32, 16, 2048), seed=12)
    ranks, p, seed, t0 = (8, 4, 16), 0.1, 99, 123457
    dec = M.Decomposition(X.shape, ranks, p)
    say("hosvd on tick-keyed sample")
    dec.sample(torch.from_numpy(X).cuda(), seed, 0, tick0=t0)
    dec.hosvd()
    assert dec.status()[0] == 0
    Xh = O.sampled_tensor_ticks(X, p, seed, t0)
    for n, A_o in enumerate(O.hosvd_factors(Xh, ranks)):
        Un = O.unfold(Xh, n)
        tol = subspace_tol(O.eigengap(Un, ranks[n]), O.davis_kahan_bound(Un, ranks[n], 2.0**-24))
        A_g = dec.factors[n].cpu().numpy()
        assert sin_theta(A_o, A_g) <= tol
        assert columns_elementwise(A_o, A_g, np.linalg.svd(Un, compute_uv=False)) <= 1.0


DEGENERATE = [
    ("empty-6x5x7", 1e-6, 1, "empty"),          # the coins keep nothing
    ("zero-tensor-6x5x7", 0.5, 2, "zero"),      # kept values are all zero
    ("nan-kept-6x5x7", 0.5, 3, "nan"),          # a kept value is NaN
]


@pytest.mark.parametrize("name,p,seed,kind", DEGENERATE, ids=[c[0] for c in DEGENERATE])
def test_degenerate_sample_sets_status_and_solver_does_nothing(name, p, seed, kind):
    """Reading R10 on the device: the sample reports MACH_EDEGENERATE where
    the oracle finds the sampled tensor zero, MACH_EINVAL where it finds a
    non-finite kept value; the layouts are still exact, and HOSVD, a sweep
    and the core leave the factors and the core untouched."""
    import torch
    from paper_0909_4969_amd import mach as M
    shape, ranks = (6, 5, 7), (2, 2, 2)
    X = _input(shape, "f32", seed)
    mask = O.sample_mask(shape, p, seed, 0).ravel()
    if kind == "zero":
        X[...] = 0.0
    if kind == "nan":
        X.reshape(-1)[np.flatnonzero(mask)[0]] = np.nan
    with pytest.raises(ValueError) as e:
        O.hosvd_factors(O.sampled_tensor(X, p, seed, 0), ranks)
    expect = M.MACH_EINVAL if kind == "nan" else M.MACH_EDEGENERATE
    assert isinstance(e.value, O.DegenerateSample) == (expect == M.MACH_EDEGENERATE)
    dec = M.Decomposition(shape, ranks, p)
    say("degenerate sample", name)
    dec.sample(torch.from_numpy(X).cuda(), seed, 0)
    st, nnz, _ = dec.status()
    assert st == expect, (st, expect)
    assert nnz == int(mask.sum())
    coo = O.sample_coo(X, p, seed, 0)
    idx, _ = dec.sw.entries("coo_l", nnz)
    np.testing.assert_array_equal(idx, coo.idx)
    h, _ = S.head_split(shape)
    MH = int(np.prod(shape[:h]))
    np.testing.assert_array_equal(dec.sw.u32("rowptr", MH + 1), S.row_pointers(coo.idx, shape, h))
    say("solver on degenerate sample", name)
    dec.hosvd()
    dec.sweep()
    dec.core()
    st, _, _ = dec.status()
    assert st == expect, (st, expect)
    for f in dec.factors:
        assert not bool(f.any())
    assert not bool(dec.G.any())


def test_maximum_size_sample_sampled_positions():
    """The largest accepted tensor, 1024 x 1024 x 2047 float32 (2^31 - 2^20
    entries, 8.6 GB, drawn on the device) at p = 0.01: Binomial kept count,
    increasing kept indices, and the mask, kept values, sum of squares and
    column layout against the oracle on sampled windows of the index."""
    import torch
    from paper_0909_4969_amd import mach as M
    shape, p, seed, win = (1024, 1024, 2047), 0.01, 77, 5
    N = int(np.prod(shape))
    g = torch.Generator(device="cuda").manual_seed(123)
    X = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32)
    say("sample maximum size", shape)
    sw = M.sample(X, p, seed, win)
    st, nnz, ss = sw.status()
    assert st == 0, st
    q = O.keep_threshold(p) / 2**32
    assert abs(nnz - N * q) < 6 * math.sqrt(N * q * (1 - q))
    idx, val = sw.entries("coo_l", nnz)
    assert np.all(np.diff(idx.astype(np.int64)) > 0)
    flat = X.view(-1)
    kept_x = flat[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy()
    np.testing.assert_array_equal(val.view(np.uint32), kept_x.view(np.uint32))
    assert abs(ss - float(np.sum(kept_x.astype(np.float64) ** 2))) <= 1e-10 * ss
    rng = np.random.default_rng(2)
    starts = [0, N - 65536] + [int(s) for s in rng.integers(0, N - 65536, 6)]
    for lo in starts:
        hi = lo + 65536
        lin = np.arange(lo, hi, dtype=np.uint64)
        keep = O.mask_words(lin, seed, win).astype(np.uint64) < np.uint64(O.keep_threshold(p))
        want = np.flatnonzero(keep).astype(np.int64) + lo
        sel = (idx >= lo) & (idx < hi)
        np.testing.assert_array_equal(idx[sel].astype(np.int64), want)
    h, perm = S.head_split(shape)
    MH = int(np.prod(shape[:h]))
    order, colptr = S.column_order(idx, shape, h, perm)
    np.testing.assert_array_equal(sw.u32("colptr", N // MH + 1), colptr)
    np.testing.assert_array_equal(sw.u32("rowptr", MH + 1), S.row_pointers(idx, shape, h))
    tidx, _ = sw.entries("coo_t", nnz)
    np.testing.assert_array_equal(tidx, idx[order])

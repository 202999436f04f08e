"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function include/mach.h declares, and its host logic (size queries, layout
choice, argument checks, status strings, built-in self test) behaves; no
call here launches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mach.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mach_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def M():
    from paper_0909_4969_amd import mach
    return mach


def test_library_exports_every_declared_function(M):
    lib = ctypes.CDLL(M._LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mach.h but not exported"
    assert sorted(M.EXPORTED) == names


def test_host_selftest(M):
    assert M.host_selftest() == 0


def test_status_strings(M):
    for code in (M.MACH_OK, M.MACH_EINVAL, M.MACH_ENOMEM, M.MACH_EDEVICE, M.MACH_EUNSUPPORTED,
                 M.MACH_EDEGENERATE, M.MACH_ENOCONV):
        assert M.status_string(code)
    assert M.status_string(-99)


def test_gram_free_tail_hosvd_reserves_no_gram(M):
    # 48 x 48 = 2304 head rows, more than the sparse tail Gram holds: the
    # tail mode's HOSVD Gram (2304^2 float64) is never formed, so this window
    # needs less solver workspace than a smaller one with 2016 head rows,
    # whose 2016^2 Gram (32.5 MB) is reserved in each of its two lanes
    ranks = (8, 8, 16)
    formed = M.solver_workspace_bytes((48, 42, 4096), ranks, 1000)
    gram_free = M.solver_workspace_bytes((48, 48, 4096), ranks, 1000)
    assert formed > 0 and gram_free > 0
    assert gram_free < formed


def test_size_queries(M):
    shape, ranks = (128, 16, 16384), (8, 4, 16)
    cap = M.nnz_capacity(shape, 0.1)
    N = 128 * 16 * 16384
    assert 0.1 * N < cap < 0.1 * N + 10 * (N * 0.09) ** 0.5 + 1024
    assert M.nnz_capacity(shape, 1.0) >= N
    sb = M.sample_workspace_bytes(shape, cap)
    assert sb >= 8 * cap * 2 + N // 8
    assert M.solver_workspace_bytes(shape, ranks, cap) > 0
    assert M.solver_workspace_bytes(shape, ranks, cap, M.MACH_BF16) > 0
    assert M.solver_workspace_bytes(shape, ranks, cap, M.MACH_FP8E4M3) > 0
    assert M.solver_workspace_bytes(shape, ranks, cap, M.MACH_F64) == 0
    # invalid: rank above the dimension, above 16, too many modes, empty mode
    assert M.solver_workspace_bytes((8, 8, 8), (9, 2, 2), 100) == 0
    assert M.solver_workspace_bytes((64, 64, 64), (17, 2, 2), 100) == 0
    assert M.solver_workspace_bytes((4, 4, 4, 4, 4), (2, 2, 2, 2, 2), 100) == 0
    assert M.sample_workspace_bytes((4, 0, 4), 10) == 0
    # the largest tensor: fewer than 2^31 entries (uint32 linear indices with
    # headroom for the word arithmetic of the coin toss)
    assert M.sample_workspace_bytes((1024, 1024, 2047), 1 << 20) > 0
    assert M.sample_workspace_bytes((1024, 1024, 2048), 1 << 20) == 0
    assert M.nnz_capacity((1024, 1024, 2048), 0.01) == 0


def test_layout_choice(M):
    for shape in ((128, 16, 16384), (64, 32, 48), (16, 16, 16, 64), (300, 200)):
        h, perm = M.layout_info(shape)
        d = len(shape)
        assert 1 <= h < d and d - h <= 2 and h <= 2
        assert sorted(perm) == list(range(h))
        if h == 2:   # the larger head mode innermost
            assert shape[perm[1]] >= shape[perm[0]]


def test_sample_offsets_are_disjoint_and_aligned(M):
    shape = (128, 16, 16384)
    cap = M.nnz_capacity(shape, 0.1)
    import ctypes as C
    out = (C.c_uint64 * 6)()
    rc = M.LIB.mach_sample_offsets(C.byref(M.Shape.of(shape)), cap, out, 6)
    assert rc == M.MACH_OK
    offs = sorted(int(x) for x in out)
    assert all(o % 256 == 0 for o in offs)
    assert len(set(offs)) == 6
    assert offs[-1] < M.sample_workspace_bytes(shape, cap)


def test_timing_hook_host_side(M):
    """Sampling choice of the kernel timing hook (host state only)."""
    import ctypes as C
    assert M.LIB.mach_timing_enable(-1) == M.MACH_EINVAL
    assert M.LIB.mach_timing_enable(10) == M.MACH_OK
    ms, n = C.c_double(-1.0), C.c_int32(-1)
    assert M.LIB.mach_timing_read(0, C.byref(ms), C.byref(n)) == M.MACH_OK
    assert n.value == 0 and ms.value == 0.0
    assert M.LIB.mach_timing_read(2, C.byref(ms), C.byref(n)) == M.MACH_EINVAL
    assert M.LIB.mach_timing_enable(0) == M.MACH_OK


def test_sample_ticks_rejects_wrapping_ticks(M):
    """Host-side argument checks of mach_sample_ticks (no launch happens)."""
    import ctypes as C
    shape = (4, 8)
    s = M.Shape.of(shape)
    cap = M.nnz_capacity(shape, 0.5)
    fake = C.c_void_p(1 << 20)          # aligned; never dereferenced on these paths
    nb = M.sample_workspace_bytes(shape, cap)
    rc = M.LIB.mach_sample_ticks(C.byref(s), M.MACH_F32, fake, 0.5, 1, (1 << 64) - 4, fake, nb, cap, None)
    assert rc == M.MACH_EINVAL
    rc = M.LIB.mach_sample_ticks(C.byref(s), M.MACH_F32, fake, 1.5, 1, 0, fake, nb, cap, None)
    assert rc == M.MACH_EINVAL
    rc = M.LIB.mach_sample_ticks(C.byref(s), M.MACH_F32, fake, 0.5, 1, 0, fake, nb - 1, cap, None)
    assert rc == M.MACH_ENOMEM


def test_layout_split_follows_the_stated_rule(M):
    """mach_layout_info agrees with the rule stated in the segment oracle
    (which the GPU layout tests use instead of asking the library)."""
    from oracle import segments as S
    shapes = [(128, 16, 16384), (64, 32, 48), (16, 16, 16, 64), (300, 200), (37, 53), (5, 7, 9),
              (3, 5, 7, 11), (64, 64, 64, 256), (96, 12, 12), (600, 12, 12), (16, 16, 16, 256),
              (1024, 1024, 2047), (7, 5, 333), (4, 4, 4, 97), (2, 3, 4, 5, 6), (3, 3, 3, 3, 3, 3),
              (9, 2), (2, 9), (8, 8, 8, 8), (1, 5, 7), (96, 80, 6), (6, 5, 7)]
    for shape in shapes:
        assert M.layout_info(shape) == S.head_split(shape), shape



def test_tucker2_layout_rules(M):
    """An uncompressed last mode (rank 0) is accepted when it is the single
    tail mode and every other mode's Gram is on the row side."""
    assert M.solver_workspace_bytes((128, 16, 16384), (8, 4, 0), 1000) > 0
    assert M.solver_workspace_bytes((54, 4, 5385), (5, 2, 0), 1000) > 0
    assert M.solver_workspace_bytes((200, 300), (6, 0), 1000) > 0
    # two tail modes, a column-side mode, a zero rank elsewhere
    assert M.solver_workspace_bytes((64, 64, 64, 256), (10, 10, 10, 0), 1000) == 0
    assert M.solver_workspace_bytes((600, 12, 12), (10, 10, 0), 1000) == 0
    assert M.solver_workspace_bytes((128, 16, 16384), (0, 4, 16), 1000) == 0
    # the workspace holds the dense sampled tensor
    assert M.solver_workspace_bytes((128, 16, 16384), (8, 4, 0), 1000) >= 4 * 128 * 16 * 16384

"""Python binding of libmach.so (include/mach.h).

Argument marshalling only: every step of the MACH path runs in the HIP
kernels of the library.  Device memory comes from torch (plain uint8 /
float64 tensors on a CUDA device); the current torch stream is passed as
the hipStream_t.  Importing this module fails loudly if the library is
missing or was not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmach.so")

MACH_OK, MACH_EINVAL, MACH_ENOMEM, MACH_EDEVICE = 0, -1, -2, -3
MACH_EUNSUPPORTED, MACH_EDEGENERATE, MACH_ENOCONV = -4, -5, -6
MACH_F64, MACH_F32, MACH_BF16, MACH_FP8E4M3 = 0, 1, 2, 3
MAX_D = 8

EXPORTED = (
    "mach_sample_workspace_bytes", "mach_nnz_capacity", "mach_sample", "mach_sample_ticks",
    "mach_solver_workspace_bytes", "mach_hosvd", "mach_hooi_sweep", "mach_core",
    "mach_solver_reset", "mach_layout_info", "mach_sample_offsets",
    "mach_read_status", "mach_status_string", "mach_host_selftest",
    "mach_timing_enable", "mach_timing_read", "mach_core_noalloc", "mach_sample_ticks_slide",
)


class MachError(RuntimeError):
    def __init__(self, where, code):
        self.code = code
        super().__init__(f"{where}: status {code} ({status_string(code)})")


class Shape(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("pad_", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_D)]

    @classmethod
    def of(cls, dims):
        dims = tuple(int(x) for x in dims)
        s = cls()
        s.d = len(dims)
        for i, v in enumerate(dims):
            s.dims[i] = v
        return s


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_0909_4969_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, U64, I32, SZ, D = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
    SP = ctypes.POINTER(Shape)
    IP = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "mach_sample_workspace_bytes": (SZ, [SP, U64]),
        "mach_nnz_capacity": (U64, [SP, D]),
        "mach_sample": (I32, [SP, I32, P, D, U64, U64, P, SZ, U64, P]),
        "mach_sample_ticks": (I32, [SP, I32, P, D, U64, U64, P, SZ, U64, P]),
        "mach_sample_ticks_slide": (I32, [SP, I32, P, D, U64, U64, P, P, SZ, U64, P]),
        "mach_solver_workspace_bytes": (SZ, [SP, IP, I32, U64]),
        "mach_hosvd": (I32, [P, U64, SP, IP, P, P, SZ, P]),
        "mach_hooi_sweep": (I32, [P, U64, SP, IP, P, I32, I32, P, SZ, P, P]),
        "mach_core": (I32, [P, U64, SP, IP, P, P, P, P, SZ, P]),
        "mach_core_noalloc": (I32, [P, U64, SP, IP, P, P, P, P]),
        "mach_solver_reset": (I32, [SP, IP, P, SZ, P]),
        "mach_layout_info": (I32, [SP, IP, IP]),
        "mach_sample_offsets": (I32, [SP, U64, ctypes.POINTER(U64), I32]),
        "mach_read_status": (I32, [P, P, P, IP, ctypes.POINTER(U64), ctypes.POINTER(D)]),
        "mach_status_string": (ctypes.c_char_p, [I32]),
        "mach_host_selftest": (I32, []),
        "mach_timing_enable": (I32, [I32]),
        "mach_timing_read": (I32, [I32, ctypes.POINTER(D), IP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def status_string(code: int) -> str:
    return LIB.mach_status_string(int(code)).decode()


def _check(where, rc):
    if rc != MACH_OK:
        raise MachError(where, rc)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ranks(ranks):
    arr = (ctypes.c_int32 * len(ranks))(*[int(r) for r in ranks])
    return arr


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[t.data_ptr() if t is not None and t.numel() else None
                                              for t in tensors])
    return arr


def nnz_capacity(shape, p) -> int:
    return int(LIB.mach_nnz_capacity(ctypes.byref(Shape.of(shape)), float(p)))


def sample_workspace_bytes(shape, cap) -> int:
    return int(LIB.mach_sample_workspace_bytes(ctypes.byref(Shape.of(shape)), int(cap)))


def solver_workspace_bytes(shape, ranks, cap, prec=MACH_F32) -> int:
    return int(LIB.mach_solver_workspace_bytes(ctypes.byref(Shape.of(shape)), _ranks(ranks), prec, int(cap)))


def layout_info(shape):
    h = ctypes.c_int32()
    perm = (ctypes.c_int32 * MAX_D)()
    _check("mach_layout_info", LIB.mach_layout_info(ctypes.byref(Shape.of(shape)), ctypes.byref(h), perm))
    return int(h.value), [int(perm[i]) for i in range(h.value)]


def host_selftest() -> int:
    return int(LIB.mach_host_selftest())


def timing_enable(every: int):
    """Time one sparse pass in every `every` of each kind (0: off)."""
    _check("mach_timing_enable", LIB.mach_timing_enable(int(every)))


def timing_read(which: int):
    """(total milliseconds, launches) of the sparse passes of one kind since
    timing was enabled: which = 0 head-row pass, 1 tail-column pass."""
    ms, n = ctypes.c_double(), ctypes.c_int32()
    _check("mach_timing_read", LIB.mach_timing_read(int(which), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


@dataclass
class SampleWorkspace:
    """A sample workspace on the device and what it was built for."""
    shape: tuple
    cap: int
    buf: torch.Tensor          # uint8, device

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())

    def offsets(self):
        out = (ctypes.c_uint64 * 6)()
        _check("mach_sample_offsets", LIB.mach_sample_offsets(ctypes.byref(Shape.of(self.shape)),
                                                              self.cap, out, 6))
        return dict(zip(("coo_l", "rowptr", "coo_t", "colptr", "bitmap", "wrank"), list(out)))

    def status(self, solver: torch.Tensor | None = None, stream=None):
        """Synchronises the stream; returns (status, nnz, sum of kept x^2)."""
        st, nnz, ss = ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_double()
        sp = ctypes.c_void_p(solver.data_ptr()) if solver is not None else None
        _check("mach_read_status", LIB.mach_read_status(self.ptr, sp, _stream(stream), ctypes.byref(st),
                                                        ctypes.byref(nnz), ctypes.byref(ss)))
        return int(st.value), int(nnz.value), float(ss.value)

    def entries(self, which="coo_l", nnz=None):
        """(l uint32 as int64, value float32) of the kept entries, copied to the host."""
        if nnz is None:
            nnz = self.status()[1]
        off = self.offsets()[which]
        raw = self.buf[off:off + 8 * nnz].view(torch.int32).view(-1, 2).cpu()
        idx = raw[:, 0].numpy().view("uint32").copy()
        val = raw[:, 1].numpy().view("float32").copy()
        return idx, val

    def u32(self, which, count):
        off = self.offsets()[which]
        return self.buf[off:off + 4 * count].view(torch.int32).cpu().numpy().view("uint32").copy()

    def u64(self, which, count):
        off = self.offsets()[which]
        return self.buf[off:off + 8 * count].view(torch.int64).cpu().numpy().view("uint64").copy()


def sample(X: torch.Tensor, p: float, seed: int, window_id: int, cap: int | None = None,
           ws: SampleWorkspace | None = None, stream=None, tick0: int | None = None,
           prev: SampleWorkspace | None = None) -> SampleWorkspace:
    """MACH's coin toss over the device tensor X (float32 or float64).  With
    tick0, the coins are keyed on (seed, series, absolute tick) instead of
    (seed, window_id, linear index): X's last mode holds ticks tick0, ...;
    with tick0 and prev (the sample of an earlier window of the same stream,
    shape, seed, p and capacity), the measurements the two windows share
    keep prev's coins and values (mach_sample_ticks_slide)."""
    if not X.is_cuda or not X.is_contiguous():
        raise ValueError("X must be a contiguous device tensor")
    dt = {torch.float32: MACH_F32, torch.float64: MACH_F64}.get(X.dtype)
    if dt is None:
        raise ValueError("X must be float32 or float64")
    shape = tuple(X.shape)
    if cap is None:
        cap = nnz_capacity(shape, p) if ws is None else ws.cap
    if ws is None:
        nb = sample_workspace_bytes(shape, cap)
        if nb == 0:
            raise MachError("mach_sample_workspace_bytes", MACH_EINVAL)
        ws = SampleWorkspace(shape, cap, torch.empty(nb, dtype=torch.uint8, device=X.device))
    s = Shape.of(shape)
    if prev is not None:
        if tick0 is None:
            raise ValueError("a slid window needs tick0")
        _check("mach_sample_ticks_slide",
               LIB.mach_sample_ticks_slide(ctypes.byref(s), dt, ctypes.c_void_p(X.data_ptr()), float(p),
                                           int(seed), int(tick0), prev.ptr, ws.ptr, ws.buf.numel(), cap,
                                           _stream(stream)))
        return ws
    if tick0 is not None:
        _check("mach_sample_ticks", LIB.mach_sample_ticks(ctypes.byref(s), dt, ctypes.c_void_p(X.data_ptr()),
                                                          float(p), int(seed), int(tick0), ws.ptr,
                                                          ws.buf.numel(), cap, _stream(stream)))
        return ws
    _check("mach_sample", LIB.mach_sample(ctypes.byref(s), dt, ctypes.c_void_p(X.data_ptr()), float(p),
                                          int(seed), int(window_id), ws.ptr, ws.buf.numel(), cap,
                                          _stream(stream)))
    return ws


def solver_workspace(shape, ranks, cap, device="cuda") -> torch.Tensor:
    nb = solver_workspace_bytes(shape, ranks, cap)
    if nb == 0:
        raise MachError("mach_solver_workspace_bytes", MACH_EINVAL)
    return torch.empty(nb, dtype=torch.uint8, device=device)


def _factors_ok(factors, shape, ranks):
    for A, I, R in zip(factors, shape, ranks):
        if R == 0:          # uncompressed mode (identity factor): passed as NULL
            continue
        if A.dtype != torch.float64 or not A.is_cuda or tuple(A.shape) != (I, R) or not A.is_contiguous():
            raise ValueError("factors must be contiguous float64 device tensors of shape (I_n, R_n)")


def core_shape(shape, ranks):
    """Shape of the core: R_n, or I_n for an uncompressed mode (R_n = 0)."""
    return tuple(int(r) if r > 0 else int(I) for I, r in zip(shape, ranks))


def hosvd(sw: SampleWorkspace, ranks, solver: torch.Tensor, factors=None, stream=None):
    """MACH-HOSVD factors (Alg. 1).  Returns the list of float64 factors."""
    if factors is None:
        factors = [torch.empty(I, R, dtype=torch.float64, device=sw.buf.device)
                   for I, R in zip(sw.shape, ranks)]
    _factors_ok(factors, sw.shape, ranks)
    s = Shape.of(sw.shape)
    _check("mach_hosvd", LIB.mach_hosvd(sw.ptr, sw.cap, ctypes.byref(s), _ranks(ranks),
                                        _ptr_array(factors), ctypes.c_void_p(solver.data_ptr()),
                                        solver.numel(), _stream(stream)))
    return factors


def solver_stats(solver: torch.Tensor):
    """Diagnostics kept in the solver workspace (synchronises), cleared by
    each HOSVD.  Per mode, for its last sweep eigensolve: the Jacobi sweeps
    (+1000 when warm-started, +2000 when warm-started in the rotated
    column-side basis), 3000 + the Rayleigh-Ritz rounds of a block subspace
    iteration (on Y Y^T or on the Gram), or the steps of the subspace
    iteration of a larger Gram (+10000 when the residual tolerance was not
    reached); and for its HOSVD eigensolve the same codes of the block or
    subspace iteration, 0 after a Jacobi solve."""
    raw = solver[96:160].view(torch.int32).cpu().tolist()
    return {"jacobi_sweeps": raw[:8], "hosvd_subspace_steps": raw[8:16]}


def solver_reset(shape, ranks, solver: torch.Tensor, stream=None):
    _check("mach_solver_reset", LIB.mach_solver_reset(ctypes.byref(Shape.of(shape)), _ranks(ranks),
                                                      ctypes.c_void_p(solver.data_ptr()), solver.numel(),
                                                      _stream(stream)))


def hooi_sweep(sw: SampleWorkspace, ranks, factors, solver: torch.Tensor, first_mode=0,
               fit: torch.Tensor | None = None, prec=MACH_F32, stream=None):
    """One HOOI sweep (Alg. 2) over modes first_mode..d-1, updating `factors` in place."""
    _factors_ok(factors, sw.shape, ranks)
    s = Shape.of(sw.shape)
    fp = ctypes.c_void_p(fit.data_ptr()) if fit is not None else None
    _check("mach_hooi_sweep", LIB.mach_hooi_sweep(sw.ptr, sw.cap, ctypes.byref(s), _ranks(ranks),
                                                  _ptr_array(factors), prec, int(first_mode),
                                                  ctypes.c_void_p(solver.data_ptr()), solver.numel(),
                                                  fp, _stream(stream)))
    return factors


def core(sw: SampleWorkspace, ranks, factors, solver: torch.Tensor, G=None, norm2=None, stream=None):
    """G = Xhat x_n A^(n)T (eq. eqcore) as a float64 device tensor, and ||G||^2."""
    _factors_ok(factors, sw.shape, ranks)
    dev = sw.buf.device
    if G is None:
        G = torch.empty(core_shape(sw.shape, ranks), dtype=torch.float64, device=dev)
    if norm2 is None:
        norm2 = torch.empty(1, dtype=torch.float64, device=dev)
    s = Shape.of(sw.shape)
    _check("mach_core", LIB.mach_core(sw.ptr, sw.cap, ctypes.byref(s), _ranks(ranks), _ptr_array(factors),
                                      ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(norm2.data_ptr()),
                                      ctypes.c_void_p(solver.data_ptr()), solver.numel(), _stream(stream)))
    return G, norm2


def core_noalloc(sw: SampleWorkspace, ranks, factors, G: torch.Tensor, norm2: torch.Tensor, stream=None):
    """mach_core_noalloc: the core into the caller's G and norm2, with the
    library's fixed device scratch instead of a solver workspace (nothing is
    allocated by the call)."""
    _factors_ok(factors, sw.shape, ranks)
    s = Shape.of(sw.shape)
    _check("mach_core_noalloc", LIB.mach_core_noalloc(sw.ptr, sw.cap, ctypes.byref(s), _ranks(ranks),
                                                      _ptr_array(factors), ctypes.c_void_p(G.data_ptr()),
                                                      ctypes.c_void_p(norm2.data_ptr()), _stream(stream)))
    return G, norm2


class Decomposition:
    """MACH-HOOI on one device tensor: sample, HOSVD init, sweeps, core.

    All buffers are allocated once here (torch device memory); each step
    enqueues HIP kernels on the current stream."""

    def __init__(self, shape, ranks, p, device="cuda", cap=None):
        self.shape = tuple(int(x) for x in shape)
        self.ranks = tuple(int(r) for r in ranks)
        self.p = float(p)
        self.cap = int(cap) if cap is not None else nnz_capacity(self.shape, p)
        nb = sample_workspace_bytes(self.shape, self.cap)
        self.sw = SampleWorkspace(self.shape, self.cap, torch.empty(nb, dtype=torch.uint8, device=device))
        self.solver = solver_workspace(self.shape, self.ranks, self.cap, device)
        self.factors = [torch.zeros(I, R, dtype=torch.float64, device=device)
                        for I, R in zip(self.shape, self.ranks)]
        self.fit = torch.zeros(1, dtype=torch.float64, device=device)
        self.G = torch.zeros(core_shape(self.shape, self.ranks), dtype=torch.float64, device=device)
        self.norm2 = torch.zeros(1, dtype=torch.float64, device=device)

    def sample(self, X, seed, window_id, stream=None, tick0=None, prev=None):
        sample(X, self.p, seed, window_id, ws=self.sw, stream=stream, tick0=tick0, prev=prev)

    def hosvd(self, stream=None):
        hosvd(self.sw, self.ranks, self.solver, self.factors, stream=stream)

    def sweep(self, first_mode=0, prec=MACH_F32, stream=None):
        hooi_sweep(self.sw, self.ranks, self.factors, self.solver, first_mode, self.fit, prec, stream)

    def core(self, stream=None):
        core(self.sw, self.ranks, self.factors, self.solver, self.G, self.norm2, stream)
        return self.G

    def status(self, stream=None):
        return self.sw.status(self.solver, stream)

    def run(self, X, seed, window_id, sweeps, stream=None):
        self.sample(X, seed, window_id, stream)
        self.hosvd(stream)
        for _ in range(sweeps):
            self.sweep(stream=stream)
        self.core(stream)
        return self

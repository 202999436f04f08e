"""Shared helpers of the GPU parity tests (host side only)."""
import math
import sys

import numpy as np

from oracle import mach as O


def say(*a):
    """Names the case before each GPU step, flushed."""
    print(*a, flush=True)
    sys.stdout.flush()


def pack_mask(mask_flat: np.ndarray, nwords: int) -> np.ndarray:
    bits = np.zeros(nwords * 64, dtype=bool)
    bits[:mask_flat.size] = mask_flat
    return np.packbits(bits, bitorder="little").view("<u8")


def oracle_sweep_with_gaps(Xh, factors, ranks, first_mode=0):
    """One oracle HOOI sweep that also returns, per updated mode, the
    relative eigengap and the Davis-Kahan FP32 bound of Y_(n)."""
    A = [np.array(a, dtype=np.float64) for a in factors]
    gaps, dk = {}, {}
    for n in range(first_mode, Xh.ndim):
        Yn = O.unfold(O.ttm_chain(Xh, A, n), n)
        gaps[n] = O.eigengap(Yn, ranks[n])
        dk[n] = O.davis_kahan_bound(Yn, ranks[n], 2.0 ** -24)
        A[n] = O.leading_left_singular_vectors(Yn, ranks[n])[0]
    return A, gaps, dk


def subspace_tol(gap, dk, base=1e-5):
    """1e-5 where the eigengap is healthy (>= 1e-3); otherwise the stated
    Davis-Kahan bound (never below 1e-5)."""
    return base if gap >= 1e-3 else max(base, min(1.0, 4.0 * dk))


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

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


# Measures applied to what the device returned.  They never go through the
# oracle: the oracle only ever sees host inputs and its own results.

def sin_theta(A_ref, A):
    """Sine of the largest principal angle between span(A_ref) and span(A),
    ||(I - A_ref A_ref^T) A||_2, for orthonormal bases."""
    A_ref = np.asarray(A_ref, np.float64)
    A = np.asarray(A, np.float64)
    P = A - A_ref @ (A_ref.T @ A)
    return float(np.linalg.norm(P, 2)) if P.size else 0.0


def project(T, factors):
    """T x_1 A_1^T x_2 ... x_d A_d^T in float64 (the mode products spelled
    out with tensordot; mode n of the result has size R_n)."""
    R = np.asarray(T, np.float64)
    for n, A in enumerate(factors):
        R = np.moveaxis(np.tensordot(np.asarray(A, np.float64), R, axes=(0, n)), 0, n)
    return R


def recon_rel_error(X, G, factors):
    """||X - G x_n A_n|| / ||X|| for orthonormal factors, from
    ||X||^2 - 2 <X x_n A_n^T, G> + ||G||^2."""
    X = np.asarray(X, np.float64)
    G = np.asarray(G, np.float64)
    nx2 = float(np.sum(X * X))
    val = nx2 - 2.0 * float(np.sum(project(X, factors) * G)) + float(np.sum(G * G))
    return math.sqrt(max(0.0, val) / nx2)


def load_factors(dec, factors):
    """Copies host float64 factors into a decomposition's device factors, so
    that a device step and an oracle step start from the same input."""
    import torch
    for f, a in zip(dec.factors, factors):
        f.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)))

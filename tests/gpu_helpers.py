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


def oracle_sweep_with_gaps(Xh, factors, ranks, first_mode=0, sing=None):
    """One oracle HOOI sweep that also returns, per updated mode, the
    relative eigengap and the Davis-Kahan FP32 bound of Y_(n); with a dict
    `sing`, also the singular values of each Y_(n) in it."""
    A = [np.array(a, dtype=np.float64) if a is not None else None for a in factors]
    gaps, dk = {}, {}
    for n in range(first_mode, Xh.ndim):
        if ranks[n] == 0:       # uncompressed mode: identity, not updated
            continue
        Yn = O.unfold(O.ttm_chain(Xh, A, n), n)
        gaps[n] = O.eigengap(Yn, ranks[n])
        dk[n] = O.davis_kahan_bound(Yn, ranks[n], 2.0 ** -24)
        A[n], s = O.leading_left_singular_vectors(Yn, ranks[n])
        if sing is not None:
            sing[n] = s
    return A, gaps, dk


def spectrum(M):
    """Singular values of M (descending) from the eigenvalues of its
    smaller-side Gram in float64: a fast test-side measure for very wide
    unfoldings (the oracle's own factors always come from its SVD)."""
    M = np.asarray(M, np.float64)
    G = M @ M.T if M.shape[0] <= M.shape[1] else M.T @ M
    w = np.linalg.eigvalsh(G)[::-1]
    return np.sqrt(np.clip(w, 0.0, None))


def gap_and_dk(s, r, u=2.0 ** -24):
    """From singular values s: the relative eigengap (lambda_r - lambda_{r+1})
    / lambda_1 of the Gram and the Davis-Kahan bound 4 u sum(lambda) /
    (lambda_r - lambda_{r+1}), as the oracle's eigengap and
    davis_kahan_bound compute them from the matrix."""
    lam = np.concatenate([np.asarray(s, np.float64) ** 2, np.zeros(max(0, r + 1 - len(s)))])
    gap = lam[r - 1] - lam[r]
    rel_gap = float(gap / lam[0]) if lam[0] > 0 else 0.0
    dk = float("inf") if gap <= 0 else float(4 * u * lam.sum() / gap)
    return rel_gap, dk


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
        if A is None:       # uncompressed mode: identity
            continue
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
        if a is None:       # uncompressed mode: no device factor
            continue
        f.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)))


def columns_elementwise(A_ref, A, s, u=2.0 ** -24, base=1e-5):
    """Column by column, entry by entry: each column of A obeys the sign
    rule (its entry of largest magnitude is positive, up to a tie within
    1e-6), and where the eigenvalue lambda_i = s_i^2 of that column is
    separated from its neighbours by g_i, the entries agree with A_ref's
    within max(1e-5, 4 u sum(s^2) / g_i) (1e-5 alone when g_i >= 1e-3
    lambda_1): the Davis-Kahan bound for one eigenvector.  The comparison
    aligns the sign first, so a tie in the sign rule is not counted twice.
    Returns the worst ratio of difference to bound (<= 1 passes)."""
    A_ref = np.asarray(A_ref, np.float64)
    A = np.asarray(A, np.float64)
    lam = np.asarray(s, np.float64) ** 2
    worst = 0.0
    for i in range(A.shape[1]):
        col = A[:, i]
        mags = np.abs(col)
        k = int(np.argmax(mags))
        assert col[k] > 0 or np.sum(mags >= mags[k] * (1 - 1e-6)) > 1, ("sign rule", i)
        left = lam[i - 1] - lam[i] if i > 0 else np.inf
        right = lam[i] - lam[i + 1] if i + 1 < lam.size else lam[i]
        g = min(left, right)
        if g >= 1e-3 * lam[0]:
            tol = base
        else:
            tol = max(base, min(2.0, 4.0 * u * float(lam.sum()) / g)) if g > 0 else 2.0
        sg = 1.0 if float(col @ A_ref[:, i]) >= 0 else -1.0
        worst = max(worst, float(np.abs(sg * col - A_ref[:, i]).max()) / tol)
    return worst

"""FP64 oracle of MACH-HOSVD / MACH-HOOI.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product path.

Everything here runs in float64 on the CPU, one step at a time, in the order
and notation of the paper.  Citations are to the paper's sections, equations
and algorithms:
  * Section 2.1 "Tensor Concepts": the norm (eq. norm), the inner product,
    matricization (the index map I_k x prod_{j!=k} I_j), the n-mode product,
    its commutativity, same-mode composition (eq. eqb) and norm invariance
    (eq. eqa).
  * Section 2.1 "Tucker3 Algorithms": HOSVD factors are leading left singular
    vectors of each matricization; the core is eq. eqcore; HOOI alternates
    one mode at a time.
  * Theorem 1 and Remark 1: the sampled tensor keeps X/p with probability p.
  * Algorithm 1 (MACH-HOSVD) and Algorithm 2 (MACH-HOOI).

Readings where the paper is silent or ambiguous:
  R1  Factors come from the sampled tensor X-hat (Alg. 1), not X.
  R2  One coin per entry, zero entries included; the coin is Philox4x32-10
      keyed by (seed, window) on the C-order linear index (oracle/philox.py);
      keep iff word < T with T = min(2^32, floor(p * 2^32)).
  R3  Singular vectors: descending singular values; in each column the entry
      of largest magnitude is made positive (ties: lowest row).
  R4  HOOI updates modes in order 1..d, each update seen by the next (the
      inner FOR of Alg. 2).  A sweep may start at a later mode (warm start).
  R5  "Fit stops improving" has no tolerance in the paper: a fixed number of
      sweeps is run and the fit is reported after every sweep.
  R6  Norm invariance (eq. eqa) holds for U with orthonormal columns
      (U^T U = I); the paper writes U U^T = I.
  R9  Streams (Remark 2: a coin as each measurement arrives): for a window
      whose last mode is time, the coin of a measurement is keyed by (seed,
      series, absolute tick) -- Philox4x32-10 at counter (tick/4 lo, tick/4
      hi, series, 0), word tick mod 4 -- so every window that contains the
      measurement draws the same coin (oracle/philox.py, mask_words_ticks).
  R10 A sampled tensor with no nonzero entry (nothing kept, or X zero where
      kept) has zero matricizations: their leading singular vectors, and so
      the factors of Alg. 1 and 2, are not determined.  Such a sample is
      degenerate (DegenerateSample); one with a non-finite entry is rejected
      (ValueError).
  R11 Tucker-n (Section 2.1: compressing n of the d modes): a mode given
      rank 0 is not compressed; its factor is the identity (None here), HOOI
      does not update it, and the core keeps that mode's full size.  HOSVD
      and HOOI of the other modes are unchanged (Alg. 1/2 with the identity
      in the products).

Parity status: every function below is pinned by tests/test_oracle_*.py,
except `theorem1_hypotheses` (report-only: its conditions are checked, the
bound is not asserted).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .philox import mask_words, mask_words_ticks

# ---------------------------------------------------------------------------
# Sampling (Theorem 1; Remark 1; Alg. 1 and Alg. 2, "MACH" block)
# ---------------------------------------------------------------------------


def keep_threshold(p: float) -> int:
    """Integer threshold T: an entry is kept iff its 32-bit word is < T.

    T = min(2^32, floor(p * 2^32)), computed in float64 (p * 2^32 is exact).
    The realised keep probability is T / 2^32, within 2^-32 of p."""
    if not (0.0 < p <= 1.0):
        raise ValueError("p must lie in (0, 1]")
    return min(1 << 32, int(math.floor(p * 4294967296.0)))


def sample_mask(shape, p: float, seed: int, window_id: int) -> np.ndarray:
    """Boolean keep-mask over a C-order tensor of `shape` (reading R2)."""
    n = int(np.prod(shape))
    T = keep_threshold(p)
    out = np.empty(n, dtype=bool)
    step = 1 << 22
    for s in range(0, n, step):
        lin = np.arange(s, min(n, s + step), dtype=np.uint64)
        out[s:s + lin.size] = mask_words(lin, seed, window_id).astype(np.uint64) < np.uint64(T)
    return out.reshape(shape)


def sample_mask_ticks(shape, p: float, seed: int, tick0: int) -> np.ndarray:
    """Boolean keep-mask of a window of a stream (reading R9): the last mode
    is time, holding ticks tick0 .. tick0 + shape[-1] - 1; the coin of entry
    (series j, tick tau) depends on (seed, j, tau) only."""
    T = int(shape[-1])
    nser = int(np.prod(shape[:-1]))
    thr = np.uint64(keep_threshold(p))
    out = np.empty((nser, T), dtype=bool)
    ticks = np.uint64(tick0) + np.arange(T, dtype=np.uint64)
    step = max(1, (1 << 22) // T)
    for j0 in range(0, nser, step):
        js = np.arange(j0, min(nser, j0 + step), dtype=np.uint64)[:, None]
        out[j0:j0 + js.shape[0]] = mask_words_ticks(js, ticks[None, :], seed).astype(np.uint64) < thr
    return out.reshape(shape)


def sample_coo_ticks(X: np.ndarray, p: float, seed: int, tick0: int) -> SampledCOO:
    """The coin toss of a stream window with tick-keyed coins, as a COO list."""
    if X.size >= (1 << 32):
        raise ValueError("linear indices must fit in 32 bits")
    mask = sample_mask_ticks(X.shape, p, seed, tick0).ravel()
    idx = np.flatnonzero(mask).astype(np.uint32)
    x = X.ravel()[idx]
    return SampledCOO(tuple(X.shape), p, idx, x.astype(np.float32),
                      float(np.sum(x.astype(np.float64) ** 2)))


def sampled_tensor_ticks(X: np.ndarray, p: float, seed: int, tick0: int) -> np.ndarray:
    """Dense X-hat of a stream window under tick-keyed coins (float64)."""
    mask = sample_mask_ticks(X.shape, p, seed, tick0)
    return np.where(mask, X.astype(np.float64) / p, 0.0)


@dataclass
class SampledCOO:
    """The kept entries in C-order linear-index order.

    idx    uint32 linear index of every kept entry (ascending)
    val    the kept input values cast to float32, NOT divided by p
    sumsq  sum of the kept values squared, float64, NOT divided by p^2
    """
    shape: tuple
    p: float
    idx: np.ndarray
    val: np.ndarray
    sumsq: float

    @property
    def nnz(self) -> int:
        return int(self.idx.size)

    @property
    def norm2_xhat(self) -> float:
        """||X-hat||^2 = sum (x/p)^2 over kept entries (eq. norm)."""
        return self.sumsq / (self.p * self.p)


def sample_coo(X: np.ndarray, p: float, seed: int, window_id: int) -> SampledCOO:
    """MACH's coin toss over every entry of X (Alg. 1/2), as a COO list."""
    if X.size >= (1 << 32):
        raise ValueError("linear indices must fit in 32 bits")
    mask = sample_mask(X.shape, p, seed, window_id).ravel()
    idx = np.flatnonzero(mask).astype(np.uint32)
    x = X.ravel()[idx]
    return SampledCOO(tuple(X.shape), p, idx, x.astype(np.float32),
                      float(np.sum(x.astype(np.float64) ** 2)))


def sampled_tensor(X: np.ndarray, p: float, seed: int, window_id: int) -> np.ndarray:
    """Dense X-hat in float64: X/p where the coin kept the entry, else 0."""
    mask = sample_mask(X.shape, p, seed, window_id)
    return np.where(mask, X.astype(np.float64) / p, 0.0)


def dense_from_coo(coo: SampledCOO, scale_by_p: bool = True) -> np.ndarray:
    """X-hat rebuilt from the COO list, float64 (values / p if scale_by_p)."""
    out = np.zeros(int(np.prod(coo.shape)), dtype=np.float64)
    v = coo.val.astype(np.float64)
    out[coo.idx.astype(np.int64)] = v / coo.p if scale_by_p else v
    return out.reshape(coo.shape)


# ---------------------------------------------------------------------------
# Section 2.1: norm, inner product, matricization, n-mode product
# ---------------------------------------------------------------------------


def norm(X) -> float:
    """Frobenius norm of a d-mode tensor (eq. norm)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.sqrt(np.sum(X * X)))


def inner(X, Y) -> float:
    """<X, Y>: sum of entrywise products (Section 2.1)."""
    return float(np.sum(np.asarray(X, np.float64) * np.asarray(Y, np.float64)))


def unfold(X: np.ndarray, k: int) -> np.ndarray:
    """Matricization along mode k: I_k x prod_{j != k} I_j.

    Element (i_1..i_d) goes to row i_k and column sum_{q != k} i_q J_q with
    J_q = prod_{m < q, m != k} I_m (0-based form of Section 2.1's map): among
    the remaining modes the lowest-numbered one varies fastest."""
    X = np.asarray(X)
    return np.moveaxis(X, k, 0).reshape(X.shape[k], -1, order="F")


def unfold_loops(X: np.ndarray, k: int) -> np.ndarray:
    """The same map written element by element (tiny tensors only)."""
    X = np.asarray(X, dtype=np.float64)
    dims = X.shape
    d = len(dims)
    J = [0] * d
    for q in range(d):
        if q == k:
            continue
        J[q] = 1
        for m in range(q):
            if m != k:
                J[q] *= dims[m]
    out = np.zeros((dims[k], X.size // dims[k]))
    for ii in np.ndindex(*dims):
        col = sum(ii[q] * J[q] for q in range(d) if q != k)
        out[ii[k], col] = X[ii]
    return out


def fold(M: np.ndarray, k: int, shape) -> np.ndarray:
    """Inverse of `unfold` for a tensor of the given shape."""
    shape = tuple(shape)
    rest = shape[:k] + shape[k + 1:]
    return np.moveaxis(np.asarray(M).reshape((shape[k],) + rest, order="F"), 0, k)


def mode_product(X: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """X x_n M for M in R^{J x I_n}: entry (.., j, ..) = sum_{i_n} x(.., i_n, ..) m(j, i_n)."""
    X = np.asarray(X, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    if M.shape[1] != X.shape[n]:
        raise ValueError("mode_product: M must be J x I_n")
    return np.moveaxis(np.tensordot(X, M, axes=([n], [1])), -1, n)


def mode_product_loops(X: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """The n-mode product written as its defining sum (tiny tensors only)."""
    X = np.asarray(X, dtype=np.float64)
    shape = list(X.shape)
    J = M.shape[0]
    out_shape = shape[:n] + [J] + shape[n + 1:]
    out = np.zeros(out_shape)
    for jj in np.ndindex(*out_shape):
        s = 0.0
        for i_n in range(shape[n]):
            src = jj[:n] + (i_n,) + jj[n + 1:]
            s += X[src] * M[jj[n], i_n]
        out[jj] = s
    return out


def multi_mode_product(X, mats, skip=None, transpose=True):
    """X x_1 M_1^T ... x_d M_d^T (transpose=True), skipping mode `skip`.

    By the commutativity of products along different modes (Section 2.1)
    the order is immaterial; modes are applied in increasing order."""
    Y = np.asarray(X, dtype=np.float64)
    for k, M in enumerate(mats):
        if k == skip or M is None:
            continue
        Y = mode_product(Y, M.T if transpose else M, k)
    return Y


# ---------------------------------------------------------------------------
# Leading left singular vectors (Section 2.2, SVD) with reading R3
# ---------------------------------------------------------------------------


def sign_fix(U: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (lowest row on ties)."""
    U = np.array(U, dtype=np.float64, copy=True)
    if U.size == 0:
        return U
    rows = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[rows, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s


def leading_left_singular_vectors(M: np.ndarray, r: int):
    """Top-r left singular vectors of M (columns, descending sigma) and all
    singular values, by LAPACK SVD in float64."""
    M = np.asarray(M, dtype=np.float64)
    if r > min(M.shape):
        raise ValueError("rank exceeds the matrix dimensions")
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    return sign_fix(U[:, :r]), s


# ---------------------------------------------------------------------------
# Algorithm 1 (MACH-HOSVD) and Algorithm 2 (MACH-HOOI)
# ---------------------------------------------------------------------------


class DegenerateSample(ValueError):
    """The sampled tensor is zero, so no factor is determined (reading R10)."""


def check_sample(Xh: np.ndarray) -> None:
    """Reading R10: rejects a sampled tensor with a non-finite entry
    (ValueError) or with no nonzero entry (DegenerateSample)."""
    if not np.all(np.isfinite(Xh)):
        raise ValueError("the sampled tensor has a non-finite entry")
    if not np.any(Xh):
        raise DegenerateSample("the sampled tensor is zero")


def hosvd_factors(Xh: np.ndarray, ranks):
    """A^(i) = r_i leading left singular vectors of X-hat_(i), i = 1..d (Alg. 1).

    Tucker-n (Section 2.1: compressing n of the d modes): a mode with r_i = 0
    is left uncompressed; its factor is None, i.e. the identity, which every
    mode product here skips."""
    check_sample(Xh)
    return [leading_left_singular_vectors(unfold(Xh, i), ranks[i])[0] if ranks[i] > 0 else None
            for i in range(Xh.ndim)]


def ttm_chain(Xh: np.ndarray, factors, n: int) -> np.ndarray:
    """Y = X-hat x_1 A1^T .. x_{n-1} A_{n-1}^T x_{n+1} A_{n+1}^T .. x_d A_d^T (Alg. 2)."""
    return multi_mode_product(Xh, factors, skip=n)


def hooi_sweep(Xh: np.ndarray, factors, ranks, first_mode: int = 0):
    """One pass of Alg. 2's REPEAT body over modes first_mode..d-1 (reading R4).

    Returns (new factors, list of ||core||^2 after each mode update).  After
    the update of mode n, ||G||^2 = sum of the top r_n squared singular values
    of Y_(n) (norm invariance, eq. eqa)."""
    check_sample(Xh)
    A = [np.array(a, dtype=np.float64) if a is not None else None for a in factors]
    trace = []
    for n in range(first_mode, Xh.ndim):
        if ranks[n] == 0:        # uncompressed mode (Tucker-n): identity, not updated
            continue
        Y = ttm_chain(Xh, A, n)
        U, s = leading_left_singular_vectors(unfold(Y, n), ranks[n])
        A[n] = U
        trace.append(float(np.sum(s[:ranks[n]] ** 2)))
    return A, trace


def core(Xh: np.ndarray, factors) -> np.ndarray:
    """G = X-hat x_1 A^(1)T x_2 ... x_d A^(d)T (eq. eqcore; last line of Alg. 1/2)."""
    return multi_mode_product(Xh, factors)


def reconstruct(G: np.ndarray, factors) -> np.ndarray:
    """G x_1 A^(1) ... x_d A^(d), the Tucker model of eq. tucker without noise."""
    return multi_mode_product(G, factors, transpose=False)


def fit_from_norms(norm2_xhat: float, norm2_core: float) -> float:
    """fit = 1 - ||X-hat - G x A|| / ||X-hat||, with the residual norm^2 taken as
    ||X-hat||^2 - ||G||^2 (orthogonal projection; eq. eqa)."""
    return 1.0 - math.sqrt(max(0.0, norm2_xhat - norm2_core)) / math.sqrt(norm2_xhat)


def rel_error(X: np.ndarray, G: np.ndarray, factors) -> float:
    """||X - G x_n A^(n)|| / ||X|| against the ORIGINAL tensor X (1 - accuracy).

    Uses ||X||^2 - 2 <X x_n A^(n)T, G> + ||G||^2, exact for orthonormal A."""
    X64 = np.asarray(X, dtype=np.float64)
    nx2 = float(np.sum(X64 * X64))
    proj = multi_mode_product(X64, factors)
    val = nx2 - 2.0 * inner(proj, G) + float(np.sum(G * G))
    return math.sqrt(max(0.0, val) / nx2)


def rel_error_dense(X: np.ndarray, G: np.ndarray, factors) -> float:
    """The same error from the explicit reconstruction (small tensors)."""
    R = reconstruct(G, factors)
    return norm(np.asarray(X, np.float64) - R) / norm(X)


@dataclass
class MachResult:
    factors: list
    core: np.ndarray
    fit_trace: list = field(default_factory=list)
    core2_trace: list = field(default_factory=list)
    norm2_xhat: float = 0.0


def mach_hooi(X, ranks, p, seed, window_id, sweeps, Xh=None) -> MachResult:
    """Alg. 2 end to end: coin toss, HOSVD init, `sweeps` HOOI sweeps, core."""
    if Xh is None:
        Xh = sampled_tensor(X, p, seed, window_id)
    n2 = float(np.sum(Xh * Xh))
    A = hosvd_factors(Xh, ranks)
    fits, c2 = [], []
    for _ in range(sweeps):
        A, tr = hooi_sweep(Xh, A, ranks)
        c2.extend(tr)
        fits.append(fit_from_norms(n2, tr[-1]))
    G = core(Xh, A)
    return MachResult(A, G, fits, c2, n2)


def mach_hosvd(X, ranks, p, seed, window_id, Xh=None) -> MachResult:
    """Alg. 1 end to end: coin toss, HOSVD factors, core."""
    if Xh is None:
        Xh = sampled_tensor(X, p, seed, window_id)
    A = hosvd_factors(Xh, ranks)
    G = core(Xh, A)
    n2 = float(np.sum(Xh * Xh))
    return MachResult(A, G, [fit_from_norms(n2, float(np.sum(G * G)))], [], n2)


# ---------------------------------------------------------------------------
# Comparison metrics
# ---------------------------------------------------------------------------


def sin_theta(A_ref: np.ndarray, A: np.ndarray) -> float:
    """||(I - A_ref A_ref^T) A||_2: sine of the largest principal angle."""
    A_ref = np.asarray(A_ref, np.float64)
    A = np.asarray(A, np.float64)
    P = A - A_ref @ (A_ref.T @ A)
    return float(np.linalg.norm(P, 2)) if P.size else 0.0


def eigengap(Yn: np.ndarray, r: int) -> float:
    """Relative gap (lambda_r - lambda_{r+1}) / lambda_1 of Y_(n) Y_(n)^T."""
    s = np.linalg.svd(np.asarray(Yn, np.float64), compute_uv=False)
    lam = np.concatenate([s ** 2, np.zeros(max(0, r + 1 - s.size))])
    return float((lam[r - 1] - lam[r]) / lam[0]) if lam[0] > 0 else 0.0


def davis_kahan_bound(Yn: np.ndarray, r: int, unit_roundoff: float) -> float:
    """4 u ||Y_(n)||_F^2 / (lambda_r - lambda_{r+1}): the subspace error a
    perturbation of size u ||Y||^2 in the Gram can cause (Davis-Kahan sin-theta)."""
    s = np.linalg.svd(np.asarray(Yn, np.float64), compute_uv=False)
    lam = np.concatenate([s ** 2, np.zeros(max(0, r + 1 - s.size))])
    gap = lam[r - 1] - lam[r]
    return float("inf") if gap <= 0 else float(4 * unit_roundoff * np.sum(s ** 2) / gap)


def pearson(a, b) -> float:
    """Pearson correlation of two vectors (the paper's PC quality measure)."""
    a = np.asarray(a, np.float64) - np.mean(a)
    b = np.asarray(b, np.float64) - np.mean(b)
    return float(np.dot(a, b) / math.sqrt(np.dot(a, a) * np.dot(b, b)))


def theorem1_hypotheses(shape, p):
    """Theorem 1's conditions: I_n >= 76, I_n^2 <= prod I_j and
    p >= max_j (8 sum_{k != j} log I_k)^4 / prod_{k != j} I_k.  Report only."""
    dims = list(shape)
    N = float(np.prod(dims))
    size_ok = all(I >= 76 and I * I <= N for I in dims)
    pmin = max((8 * sum(math.log(dims[k]) for k in range(len(dims)) if k != j)) ** 4
               / (N / dims[j]) for j in range(len(dims)))
    return {"size_conditions": size_ok, "p_min": pmin, "p_ok": p >= pmin}

"""Pins for the oracle's sampling, HOSVD (Alg. 1) and HOOI (Alg. 2), CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import mach as O

# ---------------------------------------------------------------------------
# Sampling: Theorem 1's sparsifier, Remark 1
# ---------------------------------------------------------------------------


def test_threshold():
    assert O.keep_threshold(1.0) == 1 << 32
    assert O.keep_threshold(0.5) == 1 << 31
    assert O.keep_threshold(0.1) == 429496729
    for bad in (0.0, -0.1, 1.5, float("nan")):
        with pytest.raises(ValueError):
            O.keep_threshold(bad)


def test_p_one_keeps_everything():
    X = np.random.default_rng(0).standard_normal((5, 6, 7))
    coo = O.sample_coo(X, 1.0, seed=3, window_id=9)
    assert coo.nnz == X.size
    np.testing.assert_array_equal(O.sampled_tensor(X, 1.0, 3, 9), X)


@pytest.mark.parametrize("p", [0.5, 0.1, 0.01])
def test_kept_fraction_is_binomial(p):
    shape = (64, 64, 256)
    N = int(np.prod(shape))
    q = O.keep_threshold(p) / 2**32
    k = int(O.sample_mask(shape, p, seed=11, window_id=2).sum())
    z = (k - N * q) / math.sqrt(N * q * (1 - q))
    assert abs(z) < 5


def test_slices_are_uniform_chi_square():
    shape, p = (64, 32, 512), 0.1
    m = O.sample_mask(shape, p, seed=5, window_id=0)
    for axis in range(3):
        counts = m.sum(axis=tuple(a for a in range(3) if a != axis)).astype(float)
        expect = m.sum() / shape[axis]
        chi2 = float(np.sum((counts - expect) ** 2 / expect))
        dof = shape[axis] - 1
        assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


def test_masks_differ_across_seeds_and_windows():
    shape, p = (32, 32, 64), 0.1
    a = O.sample_mask(shape, p, 1, 0)
    b = O.sample_mask(shape, p, 1, 1)
    c = O.sample_mask(shape, p, 2, 0)
    N = a.size
    for u, v in ((a, b), (a, c)):
        both = int(np.sum(u & v))
        z = (both - N * p * p) / math.sqrt(N * p * p)
        assert abs(z) < 5          # independent coins: overlap ~ p^2


def test_mask_ignores_values_and_keeps_zeros():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((8, 9, 10))
    X[X < 0] = 0.0
    c1 = O.sample_coo(X, 0.3, 7, 1)
    c2 = O.sample_coo(np.ones_like(X), 0.3, 7, 1)
    np.testing.assert_array_equal(c1.idx, c2.idx)
    assert np.any(c1.val == 0)


def test_coo_contents():
    X = np.random.default_rng(4).standard_normal((7, 11, 13))
    coo = O.sample_coo(X, 0.2, 9, 4)
    assert np.all(np.diff(coo.idx.astype(np.int64)) > 0)
    np.testing.assert_array_equal(coo.val, X.ravel()[coo.idx].astype(np.float32))
    assert abs(coo.sumsq - np.sum(X.ravel()[coo.idx] ** 2)) < 1e-9
    Xh = O.sampled_tensor(X, 0.2, 9, 4)
    np.testing.assert_allclose(O.dense_from_coo(coo), Xh, rtol=1e-7, atol=0)
    assert abs(coo.norm2_xhat - np.sum(Xh ** 2)) < 1e-9 * np.sum(Xh ** 2)


def test_unbiased_over_seeds():
    """E[X-hat] = X (Theorem 1): the seed-average of <w, X-hat> for fixed random
    weights w matches <w, X> within 5 standard errors, with
    Var = sum w^2 x^2 (1-p)/p per draw."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((16, 16, 16))
    w = rng.standard_normal(X.shape)
    p, S = 0.1, 200
    vals = [O.inner(w, O.sampled_tensor(X, p, seed=s, window_id=0)) for s in range(S)]
    truth = O.inner(w, X)
    se = math.sqrt(np.sum(w * w * X * X) * (1 - p) / p / S)
    assert abs(np.mean(vals) - truth) < 5 * se


def test_planted_missing_rescale_is_caught(monkeypatch):
    """Forgetting the 1/p rescale (Alg. 1, the kept branch) breaks unbiasedness."""
    real = O.sampled_tensor

    def wrong(X, p, seed, window_id):
        return real(X, p, seed, window_id) * p

    rng = np.random.default_rng(12)
    X = rng.standard_normal((16, 16, 16)) + 1.0
    w = np.ones_like(X)
    p, S = 0.1, 50
    vals = [O.inner(w, wrong(X, p, s, 0)) for s in range(S)]
    se = math.sqrt(np.sum(X * X) * (1 - p) / p / S)
    assert abs(np.mean(vals) - O.inner(w, X)) > 5 * se


# ---------------------------------------------------------------------------
# HOSVD (Alg. 1; Section 2.1 "Tucker3 Algorithms", eq. eqcore)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,ranks", [((12, 10, 9), (3, 4, 2)), ((6, 7, 5, 8), (2, 3, 2, 3))])
def test_hosvd_exact_for_noiseless_tucker_at_p_one(shape, ranks):
    rng = np.random.default_rng(21)
    X, _, factors = synth.tucker_tensor(shape, ranks, rng)
    res = O.mach_hosvd(X, ranks, 1.0, 0, 0)
    for A, At in zip(res.factors, factors):
        assert O.sin_theta(At, A) < 1e-12
        np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-13)
    assert O.rel_error_dense(X, res.core, res.factors) < 1e-12


def test_matrix_case_matches_eigh():
    """d = 2: MACH-HOSVD factors are the top singular vectors of the sampled
    matrix.  Pinned against LAPACK's symmetric eigensolver on M M^T and the
    Eckart-Young residual sum_{i>r} sigma_i^2."""
    rng = np.random.default_rng(22)
    M = rng.standard_normal((40, 25)) @ np.diag(np.linspace(3, 0.1, 25)) @ rng.standard_normal((25, 60))
    Mh = O.sampled_tensor(M, 0.3, 1, 0)
    r = 5
    A = O.hosvd_factors(Mh, (r, r))[0]
    w, V = np.linalg.eigh(Mh @ Mh.T)
    top = V[:, np.argsort(w)[::-1][:r]]
    assert O.sin_theta(top, A) < 1e-10
    G = O.core(Mh, O.hosvd_factors(Mh, (r, r)))
    # rank-(r, r) projection of a matrix = its rank-r truncation
    resid2 = O.norm(Mh - O.reconstruct(G, O.hosvd_factors(Mh, (r, r)))) ** 2
    lam = np.sort(w)[::-1]
    assert abs(resid2 - lam[r:].sum()) < 1e-8 * lam.sum()


def test_sign_rule():
    U = np.array([[0.6, -0.8], [-0.8, -0.6]])
    F = O.sign_fix(U)
    np.testing.assert_array_equal(F, np.array([[-0.6, 0.8], [0.8, 0.6]]))
    T = O.sign_fix(np.array([[-0.5], [0.5]]))           # tie: lowest row wins
    np.testing.assert_array_equal(T, np.array([[0.5], [-0.5]]))


# ---------------------------------------------------------------------------
# HOOI (Alg. 2)
# ---------------------------------------------------------------------------


@pytest.fixture(scope="module")
def small_problem():
    X, _ = synth.workload1(shape=(20, 16, 18), ranks=(3, 3, 3), seed=31, rel_noise=0.05)
    Xh = O.sampled_tensor(X, 0.3, 7, 0)
    return X, Xh, (3, 3, 3)


def test_hooi_core_norm_non_decreasing(small_problem):
    _, Xh, ranks = small_problem
    A = O.hosvd_factors(Xh, ranks)
    prev = float(np.sum(O.core(Xh, A) ** 2))
    for _ in range(5):
        A, trace = O.hooi_sweep(Xh, A, ranks)
        for c2 in trace:
            assert c2 >= prev * (1 - 1e-12)
            prev = c2


def test_hooi_pythagoras_and_orthonormality(small_problem):
    _, Xh, ranks = small_problem
    res = O.mach_hooi(None, ranks, 0.3, 7, 0, sweeps=3, Xh=Xh)
    for A in res.factors:
        np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-13)
    G = res.core
    resid = O.norm(Xh - O.reconstruct(G, res.factors)) ** 2
    assert abs(O.norm(Xh) ** 2 - (O.norm(G) ** 2 + resid)) < 1e-10 * O.norm(Xh) ** 2
    direct_fit = 1 - math.sqrt(resid) / O.norm(Xh)
    assert abs(direct_fit - res.fit_trace[-1]) < 1e-9


def test_all_orthogonal_core_after_update(small_problem):
    """After the mode-n update, G_(n) G_(n)^T is diagonal with the top r_n
    squared singular values of Y_(n) (Section 2.1, all-orthogonality)."""
    _, Xh, ranks = small_problem
    A = O.hosvd_factors(Xh, ranks)
    for n in range(3):
        A, _ = O.hooi_sweep(Xh, A, ranks, first_mode=n) if n == 2 else (A, None)
    A, _ = O.hooi_sweep(Xh, A, ranks)
    G = O.core(Xh, A)
    Gd = O.unfold(G, 2)
    C = Gd @ Gd.T
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 1e-10 * np.abs(C).max()
    s = np.linalg.svd(O.unfold(O.ttm_chain(Xh, A, 2), 2), compute_uv=False)
    np.testing.assert_allclose(np.sort(np.diag(C))[::-1], s[:3] ** 2, rtol=1e-10)


def test_hooi_fixed_point_at_truth():
    rng = np.random.default_rng(41)
    X, _, factors = synth.tucker_tensor((10, 9, 8), (2, 3, 2), rng)
    A, _ = O.hooi_sweep(X, factors, (2, 3, 2))
    for a, t in zip(A, factors):
        assert O.sin_theta(t, a) < 1e-12


def test_hooi_on_matrix_is_svd():
    rng = np.random.default_rng(42)
    M = rng.standard_normal((30, 20))
    A = O.hosvd_factors(M, (4, 4))
    A, _ = O.hooi_sweep(M, A, (4, 4))
    U, s, Vt = np.linalg.svd(M)
    assert O.sin_theta(U[:, :4], A[0]) < 1e-10
    assert O.sin_theta(Vt[:4].T, A[1]) < 1e-10


def test_rel_error_forms_agree(small_problem):
    X, Xh, ranks = small_problem
    res = O.mach_hooi(None, ranks, 0.3, 7, 0, sweeps=2, Xh=Xh)
    assert abs(O.rel_error(X, res.core, res.factors) - O.rel_error_dense(X, res.core, res.factors)) < 1e-10


def test_warm_start_partial_sweep_order(small_problem):
    """A sweep started at mode n updates modes n..d-1 only, in order."""
    _, Xh, ranks = small_problem
    A0 = O.hosvd_factors(Xh, ranks)
    A, trace = O.hooi_sweep(Xh, A0, ranks, first_mode=2)
    assert len(trace) == 1
    np.testing.assert_array_equal(A[0], A0[0])
    np.testing.assert_array_equal(A[1], A0[1])
    Y = O.ttm_chain(Xh, A0, 2)
    U, _ = O.leading_left_singular_vectors(O.unfold(Y, 2), 3)
    np.testing.assert_array_equal(A[2], U)


def test_planted_dropped_mode_is_caught(monkeypatch, small_problem):
    """A TTM chain that forgets one contraction (Alg. 2's Y line) makes the
    per-update core norm disagree with the core computed by eq. eqcore, so
    the fit/Pythagoras pin fails."""
    _, Xh, ranks = small_problem

    def wrong(Xh, factors, n):
        mats = list(factors)
        mats[(n + 1) % len(mats)] = None
        return O.multi_mode_product(Xh, mats, skip=n)

    monkeypatch.setattr(O, "ttm_chain", wrong)
    res = O.mach_hooi(None, ranks, 0.3, 7, 0, sweeps=2, Xh=Xh)
    resid = O.norm(Xh - O.reconstruct(res.core, res.factors)) ** 2
    direct_fit = 1 - math.sqrt(resid) / O.norm(Xh)
    assert abs(direct_fit - res.fit_trace[-1]) > 1e-3


def test_harmonic_tensor_qualitative():
    """Section 4's synthetic tensor x_ijk = 1/(i+j+k), rank (4,4,4), p = 0.1.
    The printed core values and 87% accuracy do not reproduce from the garbled table;
    what does: g(1,1,1) dominates the exact core, and the leading MACH
    components correlate with the exact ones (rho >= 0.99 per mode)."""
    n, r = 200, 4
    X = synth.harmonic_tensor(n)
    ex = O.mach_hooi(X, (r, r, r), 1.0, 0, 0, sweeps=2, Xh=X)
    G = np.abs(ex.core)
    assert G[0, 0, 0] == G.max()
    assert np.partition(G.ravel(), -2)[-2] < 0.15 * G[0, 0, 0]
    mh = O.mach_hooi(X, (r, r, r), 0.1, 1, 0, sweeps=2)
    for a, b in zip(ex.factors, mh.factors):
        assert abs(O.pearson(a[:, 0], b[:, 0])) > 0.99
    # MACH's dominant core entry stays within 1% of the exact one
    assert abs(abs(mh.core[0, 0, 0]) - G[0, 0, 0]) < 0.01 * G[0, 0, 0]


def test_theorem1_conditions_fail_for_workloads():
    """Theorem 1's hypotheses do not hold for the workloads (report-only)."""
    for w in (synth.WORKLOADS[1], synth.WORKLOADS[2], synth.WORKLOADS[3]):
        h = O.theorem1_hypotheses(w.shape, w.ps[0])
        assert not h["p_ok"]


def test_degenerate_and_non_finite_samples():
    """Reading R10: with nothing nonzero kept every matricization is zero
    (all its singular values vanish) and the factors are not determined; a
    non-finite kept value is rejected; one at a dropped position is not."""
    rng = np.random.default_rng(17)
    X = rng.standard_normal((6, 5, 7))
    mask = O.sample_mask(X.shape, 1e-6, 1, 0)
    assert not mask.any()
    Xh = O.sampled_tensor(X, 1e-6, 1, 0)
    assert all(np.linalg.svd(O.unfold(Xh, n), compute_uv=False).max() == 0.0 for n in range(3))
    with pytest.raises(O.DegenerateSample):
        O.hosvd_factors(Xh, (2, 2, 2))
    with pytest.raises(O.DegenerateSample):
        O.hosvd_factors(O.sampled_tensor(np.zeros_like(X), 0.5, 2, 0), (2, 2, 2))
    mask = O.sample_mask(X.shape, 0.5, 3, 0).ravel()
    Xn = X.copy()
    Xn.ravel()[np.flatnonzero(~mask)[0]] = np.nan          # dropped by the coin
    Xh = O.sampled_tensor(Xn, 0.5, 3, 0)
    assert np.all(np.isfinite(Xh))
    O.hosvd_factors(Xh, (2, 2, 2))
    Xn.ravel()[np.flatnonzero(mask)[0]] = np.nan           # kept
    with pytest.raises(ValueError):
        O.hosvd_factors(O.sampled_tensor(Xn, 0.5, 3, 0), (2, 2, 2))
    with pytest.raises(ValueError):
        O.hooi_sweep(O.sampled_tensor(Xn, 0.5, 3, 0), [np.eye(6, 2), np.eye(5, 2), np.eye(7, 2)], (2, 2, 2))


def test_fit_from_norms_is_the_residual_of_the_projection():
    """fit_from_norms(||Xhat||^2, ||G||^2) equals 1 - ||Xhat - G x A|| / ||Xhat||
    with the reconstruction written out (orthonormal factors, eq. eqa)."""
    rng = np.random.default_rng(8)
    Xh = rng.standard_normal((9, 7, 8))
    A = [np.linalg.qr(rng.standard_normal((s, r)))[0] for s, r in zip(Xh.shape, (3, 2, 4))]
    G = np.einsum("ijk,ia,jb,kc->abc", Xh, *A)
    R = np.einsum("abc,ia,jb,kc->ijk", G, *A)
    direct = 1.0 - np.linalg.norm(Xh - R) / np.linalg.norm(Xh)
    assert O.fit_from_norms(float(np.sum(Xh ** 2)), float(np.sum(G ** 2))) == pytest.approx(direct, abs=1e-12)
    assert O.fit_from_norms(4.0, 4.0) == 1.0 and O.fit_from_norms(4.0, 0.0) == 0.0


def test_eigengap_and_davis_kahan_closed_forms():
    """On a matrix with prescribed singular values s: the relative gap is
    (s_r^2 - s_{r+1}^2) / s_1^2 and the bound 4 u sum s^2 / (s_r^2 - s_{r+1}^2);
    a repeated s_r gives a zero gap."""
    rng = np.random.default_rng(9)
    s = np.array([5.0, 4.0, 2.0, 1.0, 0.5])
    U = np.linalg.qr(rng.standard_normal((8, 5)))[0]
    V = np.linalg.qr(rng.standard_normal((6, 5)))[0]
    Mx = U @ np.diag(s) @ V.T
    for r in (1, 2, 3):
        gap = s[r - 1] ** 2 - s[r] ** 2
        assert O.eigengap(Mx, r) == pytest.approx(gap / s[0] ** 2, rel=1e-12)
        assert O.davis_kahan_bound(Mx, r, 2.0 ** -24) == pytest.approx(4 * 2.0 ** -24 * np.sum(s ** 2) / gap, rel=1e-12)
    Mt = U @ np.diag([3.0, 3.0, 1.0, 1.0, 1.0]) @ V.T
    assert O.eigengap(Mt, 1) == pytest.approx(0.0, abs=1e-14)
    assert O.eigengap(Mx, 5) == pytest.approx(s[4] ** 2 / s[0] ** 2, rel=1e-12)   # r = rank: gap to 0

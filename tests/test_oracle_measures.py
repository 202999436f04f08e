"""Pins for the comparison measures (CPU only).

The parity tests read every subspace comparison through a principal-angle
sine and the paper's principal-component comparison (Section 4) through
Pearson's correlation.  Both the oracle's versions and the test-side
versions that measure device results (tests/gpu_helpers.py) are pinned here
against closed forms and a library routine, and planted mistakes (a dropped
projection, a Frobenius instead of a spectral norm, an uncentred or
unnormalised correlation) must fail the pins."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import mach as O
from tests import gpu_helpers as H

SIN_THETAS = {"oracle": O.sin_theta, "gpu_helpers": H.sin_theta}
PEARSONS = {"oracle": O.pearson}


def _e(n, *idx):
    out = np.zeros((n, len(idx)))
    for j, i in enumerate(idx):
        out[i, j] = 1.0
    return out


def check_sin_theta(fn):
    """Raises AssertionError unless fn(A_ref, A) is the sine of the largest
    principal angle between span(A_ref) and span(A)."""
    # one dimension: span(e1) against span(cos t e1 + sin t e2) is |sin t|
    for t in (0.0, 1e-6, 0.1, 0.7, math.pi / 4, 1.3, math.pi / 2, 2.5):
        a = np.zeros((3, 1))
        a[0, 0], a[1, 0] = math.cos(t), math.sin(t)
        assert abs(fn(_e(3, 0), a) - abs(math.sin(t))) < 1e-14, ("1-D", t)
    # two dimensions with principal angles a and b: the largest one counts
    for a, b in ((0.2, 0.5), (0.5, 0.2), (1e-3, 0.0), (0.9, 0.9), (0.0, 1.1)):
        A_ref = _e(5, 0, 1)
        A = np.zeros((5, 2))
        A[0, 0], A[2, 0] = math.cos(a), math.sin(a)
        A[1, 1], A[3, 1] = math.cos(b), math.sin(b)
        assert abs(fn(A_ref, A) - max(math.sin(a), math.sin(b))) < 1e-14, ("2-D", a, b)
    # a rotation inside the subspace changes nothing; the complement is at pi/2
    rng = np.random.default_rng(0)
    A_ref, _ = np.linalg.qr(rng.standard_normal((20, 4)))
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    assert fn(A_ref, A_ref @ Q) < 1e-14
    full, _ = np.linalg.qr(np.hstack([A_ref, rng.standard_normal((20, 4))]))
    assert abs(fn(A_ref, full[:, 4:]) - 1.0) < 1e-14
    # random pairs against the library's principal angles (Bjorck-Golub)
    for k in range(6):
        A_ref, _ = np.linalg.qr(rng.standard_normal((30, 1 + k)))
        A, _ = np.linalg.qr(A_ref + 0.3 * (k + 1) * rng.standard_normal((30, 1 + k)))
        want = math.sin(float(np.max(scipy.linalg.subspace_angles(A_ref, A))))
        assert abs(fn(A_ref, A) - want) < 1e-12, ("scipy", k)
        assert abs(fn(A, A_ref) - want) < 1e-12, ("symmetric", k)


def check_pearson(fn):
    """Raises AssertionError unless fn is Pearson's correlation coefficient."""
    x = np.array([1.0, 2.0, 3.0, 4.0])
    # hand-computed: deviations (-1.5, -.5, .5, 1.5) and (-.5, -1.5, 1.5, .5),
    # cross sum 3, squares 5 and 5: r = 3/5
    assert abs(fn(x, np.array([2.0, 1.0, 4.0, 3.0])) - 0.6) < 1e-15
    assert abs(fn(np.array([1.0, -1.0, 1.0, -1.0]), np.array([1.0, 1.0, -1.0, -1.0]))) < 1e-15
    rng = np.random.default_rng(1)
    u = rng.standard_normal(50)
    assert abs(fn(u, 3.0 * u + 2.0) - 1.0) < 1e-14
    assert abs(fn(u, -0.5 * u + 7.0) + 1.0) < 1e-14
    v = rng.standard_normal(50)
    r = fn(u, v)
    assert abs(fn(10.0 * u - 4.0, 0.1 * v + 9.0) - r) < 1e-13      # affine invariance
    assert abs(r - scipy.stats.pearsonr(u, v)[0]) < 1e-13


@pytest.mark.parametrize("name", list(SIN_THETAS))
def test_sin_theta_pins(name):
    check_sin_theta(SIN_THETAS[name])


@pytest.mark.parametrize("name", list(PEARSONS))
def test_pearson_pins(name):
    check_pearson(PEARSONS[name])


def _frobenius(A_ref, A):
    P = A - A_ref @ (A_ref.T @ A)
    return float(np.linalg.norm(P))


def _no_projection(A_ref, A):
    return float(np.linalg.norm(A - A_ref, 2))


def _cosine(A_ref, A):
    return float(np.linalg.norm(A_ref.T @ A, 2))


def _wrong_block(A_ref, A):
    P = A_ref - A @ (A.T @ A_ref)
    return float(np.linalg.norm(P[:, :1], 2))


@pytest.mark.parametrize("wrong", [_frobenius, _no_projection, _cosine, _wrong_block])
def test_planted_sin_theta_mistakes_fail_the_pins(wrong):
    with pytest.raises(AssertionError):
        check_sin_theta(wrong)


def _uncentred(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(a @ b / math.sqrt((a @ a) * (b @ b)))


def _unnormalised(a, b):
    a = np.asarray(a, float) - np.mean(a)
    b = np.asarray(b, float) - np.mean(b)
    return float(a @ b / a.size)


@pytest.mark.parametrize("wrong", [_uncentred, _unnormalised])
def test_planted_pearson_mistakes_fail_the_pins(wrong):
    with pytest.raises(AssertionError):
        check_pearson(wrong)


def test_spectrum_and_gap_measures_agree_with_the_oracles():
    """The test-side spectrum (eigenvalues of the smaller Gram) and the gap
    and Davis-Kahan figures taken from it agree with the oracle's SVD-based
    eigengap and davis_kahan_bound, on wide, tall and rank-deficient
    matrices."""
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((8, 300)), rng.standard_normal((300, 8)),
            rng.standard_normal((6, 3)) @ rng.standard_normal((3, 40))]
    for M in mats:
        s_ref = np.linalg.svd(M, compute_uv=False)
        s = H.spectrum(M)
        np.testing.assert_allclose(s[:s_ref.size], s_ref, rtol=1e-10, atol=1e-6 * s_ref[0])
        for r in (1, 2, 3):
            g, dk = H.gap_and_dk(s, r)
            assert abs(g - O.eigengap(M, r)) < 1e-9
            want = O.davis_kahan_bound(M, r, 2.0 ** -24)
            assert dk == want or abs(dk - want) <= 1e-8 * want

"""Pins of the oracle's Tucker-n path (reading R11: a mode of rank 0 is left
uncompressed, identity factor), from facts that do not depend on the code
under test:
  * a noiseless tensor with exact Tucker2 structure (core R0 x R1 x I2,
    orthonormal A0, A1) at p = 1 is recovered: zero residual, exact
    subspaces, and the core equals X x_0 A0^T x_1 A1^T;
  * Tucker2 equals Tucker3 with the third rank full (I2 <= R0 R1): the third factor
    is then an orthogonal matrix Q, the first two factors and the fit agree,
    and the Tucker3 core is the Tucker2 core rotated, G3 = G2 x_2 Q^T;
  * the brute-force definition of the Tucker2 core on a tiny tensor.
A planted mistake (the uncompressed mode contracted with a truncated basis)
fails the first pin."""
import numpy as np

import synth
from oracle import mach as O


def _tucker2(shape, r0, r1, seed):
    rng = np.random.default_rng(seed)
    A0 = np.linalg.qr(rng.standard_normal((shape[0], r0)))[0]
    A1 = np.linalg.qr(rng.standard_normal((shape[1], r1)))[0]
    C = rng.standard_normal((r0, r1, shape[2]))
    return np.einsum("abt,ia,jb->ijt", C, A0, A1), A0, A1


def test_noiseless_tucker2_is_recovered_at_p1():
    X, A0, A1 = _tucker2((12, 7, 40), 3, 2, 1)
    res = O.mach_hooi(X, (3, 2, 0), 1.0, 5, 0, sweeps=3)
    assert res.factors[2] is None
    assert res.core.shape == (3, 2, 40)
    assert O.sin_theta(A0, res.factors[0]) < 1e-12
    assert O.sin_theta(A1, res.factors[1]) < 1e-12
    # fit = 1 - sqrt(||Xhat||^2 - ||G||^2) / ||Xhat||: at zero residual the
    # difference under the root is rounding, so the fit is exact to ~1e-8 only
    assert abs(res.fit_trace[-1] - 1.0) < 1e-7
    R = O.reconstruct(res.core, res.factors)
    assert np.linalg.norm(R - X) <= 1e-12 * np.linalg.norm(X)


def test_planted_truncation_of_the_uncompressed_mode_fails():
    X, A0, A1 = _tucker2((12, 7, 40), 3, 2, 1)
    res = O.mach_hooi(X, (3, 2, 0), 1.0, 5, 0, sweeps=3)
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((40, 10)))[0]
    bad = O.reconstruct(O.multi_mode_product(X, [res.factors[0], res.factors[1], Q]),
                        [res.factors[0], res.factors[1], Q])
    assert np.linalg.norm(bad - X) > 1e-3 * np.linalg.norm(X)


def test_tucker2_equals_tucker3_with_full_third_rank():
    # full third rank needs I2 <= R0 R1 (the columns of Y_(2))
    X, _ = synth.workload1(shape=(10, 8, 5), ranks=(3, 2, 4), seed=3, rel_noise=0.2)
    t2 = O.mach_hooi(X, (3, 2, 0), 0.5, 7, 0, sweeps=4)
    t3 = O.mach_hooi(X, (3, 2, 5), 0.5, 7, 0, sweeps=4)
    for n in (0, 1):
        assert O.sin_theta(t3.factors[n], t2.factors[n]) < 1e-10
    assert abs(t2.fit_trace[-1] - t3.fit_trace[-1]) < 1e-12
    Q = t3.factors[2]
    np.testing.assert_allclose(Q.T @ Q, np.eye(5), atol=1e-12)
    # align the (sign-fixed) first two factors before comparing cores
    G2 = O.core(O.sampled_tensor(X, 0.5, 7, 0), t3.factors[:2] + [None])
    np.testing.assert_allclose(t3.core, O.mode_product(G2, Q.T, 2), atol=1e-10 * np.abs(t3.core).max())


def test_tucker2_core_by_loops():
    rng = np.random.default_rng(4)
    Xh = rng.standard_normal((4, 3, 5))
    A0 = np.linalg.qr(rng.standard_normal((4, 2)))[0]
    A1 = np.linalg.qr(rng.standard_normal((3, 2)))[0]
    G = O.core(Xh, [A0, A1, None])
    ref = np.zeros((2, 2, 5))
    for a in range(2):
        for b in range(2):
            for t in range(5):
                ref[a, b, t] = sum(Xh[i, j, t] * A0[i, a] * A1[j, b] for i in range(4) for j in range(3))
    np.testing.assert_allclose(G, ref, atol=1e-12)

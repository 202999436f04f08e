"""Pins for matricization and n-mode products (Section 2.1), CPU only."""
import numpy as np
import pytest

from oracle import mach as O


@pytest.mark.parametrize("shape", [(2, 3, 4), (3, 2, 2, 5), (4, 1, 3)])
def test_unfold_matches_index_formula(shape):
    X = np.random.default_rng(1).standard_normal(shape)
    for k in range(len(shape)):
        U = O.unfold(X, k)
        assert U.shape == (shape[k], X.size // shape[k])
        np.testing.assert_array_equal(U, O.unfold_loops(X, k))
        np.testing.assert_array_equal(O.fold(U, k, shape), X)


def test_unfold_hand_example():
    """A 2x2x2 tensor with x[i,j,k] = 100 i + 10 j + k (0-based): mode-1
    columns run (j,k) = (0,0), (1,0), (0,1), (1,1) - the lowest remaining mode
    fastest, as in Section 2.1's map."""
    X = np.zeros((2, 2, 2))
    for i, j, k in np.ndindex(2, 2, 2):
        X[i, j, k] = 100 * i + 10 * j + k
    want = np.array([[0, 10, 1, 11], [100, 110, 101, 111]], dtype=float)
    np.testing.assert_array_equal(O.unfold(X, 0), want)
    want2 = np.array([[0, 100, 1, 101], [10, 110, 11, 111]], dtype=float)
    np.testing.assert_array_equal(O.unfold(X, 1), want2)


@pytest.mark.parametrize("shape", [(2, 3, 4), (3, 2, 2, 5)])
def test_mode_product_matches_definition(shape):
    rng = np.random.default_rng(2)
    X = rng.standard_normal(shape)
    for n in range(len(shape)):
        M = rng.standard_normal((3, shape[n]))
        np.testing.assert_allclose(O.mode_product(X, M, n), O.mode_product_loops(X, M, n),
                                   rtol=1e-13, atol=1e-13)
        # unfolding form: (X x_n M)_(n) = M X_(n)
        np.testing.assert_allclose(O.unfold(O.mode_product(X, M, n), n), M @ O.unfold(X, n),
                                   rtol=1e-13, atol=1e-13)


def test_mode_product_commutes_across_modes():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 4, 5))
    A, B = rng.standard_normal((2, 3)), rng.standard_normal((6, 5))
    lhs = O.mode_product(O.mode_product(X, A, 0), B, 2)
    rhs = O.mode_product(O.mode_product(X, B, 2), A, 0)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)


def test_same_mode_composition():
    """X x_m A x_m B = X x_m (B A) (eq. eqb)."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, 4, 5))
    A, B = rng.standard_normal((6, 4)), rng.standard_normal((2, 6))
    np.testing.assert_allclose(O.mode_product(O.mode_product(X, A, 1), B, 1),
                               O.mode_product(X, B @ A, 1), rtol=1e-12, atol=1e-12)


def test_norm_invariance_needs_orthonormal_columns():
    """eq. eqa holds for U with U^T U = I (reading R6).  A wide U with
    U U^T = I drops the part of X outside its row space, so the norm shrinks."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, 5, 3))
    U, _ = np.linalg.qr(rng.standard_normal((7, 5)))          # 7x5, U^T U = I
    assert np.allclose(U.T @ U, np.eye(5))
    assert abs(O.norm(O.mode_product(X, U, 1)) - O.norm(X)) < 1e-12
    W = U[:, :3].T                                              # 3x7 ... need J x I_n = ? x 5
    V, _ = np.linalg.qr(rng.standard_normal((5, 3)))           # 5x3
    Wide = V.T                                                  # 3x5, Wide Wide^T = I
    assert np.allclose(Wide @ Wide.T, np.eye(3))
    assert O.norm(O.mode_product(X, Wide, 1)) < O.norm(X) - 1e-3
    del W


def test_norm_and_inner_product():
    rng = np.random.default_rng(6)
    X, Y = rng.standard_normal((3, 4, 2)), rng.standard_normal((3, 4, 2))
    s = 0.0
    for idx in np.ndindex(3, 4, 2):
        s += X[idx] * Y[idx]
    assert abs(O.inner(X, Y) - s) < 1e-12
    assert abs(O.norm(X) ** 2 - O.inner(X, X)) < 1e-12


def test_planted_transposed_operand_is_caught(monkeypatch):
    """Using M^T's layout by mistake (contracting the wrong axis of M) must
    fail the definition pin."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((3, 3, 3))
    M = rng.standard_normal((3, 3))

    def wrong(X, M, n):
        return np.moveaxis(np.tensordot(X, M, axes=([n], [0])), -1, n)

    monkeypatch.setattr(O, "mode_product", wrong)
    assert not np.allclose(O.mode_product(X, M, 1), O.mode_product_loops(X, M, 1))


def test_planted_c_order_unfold_is_caught(monkeypatch):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((2, 3, 4))

    def wrong(X, k):
        return np.moveaxis(X, k, 0).reshape(X.shape[k], -1)   # C order columns

    monkeypatch.setattr(O, "unfold", wrong)
    assert not np.array_equal(O.unfold(X, 0), O.unfold_loops(X, 0))

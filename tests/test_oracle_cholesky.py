"""Pins of the oracle's Cholesky factorization (oracle_cholesky_lower).

  * A = L0 L0^T with a small-integer lower-triangular L0 whose diagonal is 1, 2 or 4: the
    factor with a positive diagonal is unique, and every intermediate of the elimination is an
    exact integer or power-of-two quotient (square roots of perfect squares, divisions by
    powers of two), so the oracle must return L0 exactly;
  * the strict upper triangle is neither read nor written (NaN there stays NaN, and cannot
    reach the factor);
  * a worked example: [[4, 2], [2, 5]] = [[2, 0], [1, 2]] [[2, 1], [0, 2]];
  * reals: the backward error ||A - L L^T||_F / ||A||_F of a random symmetric positive definite
    matrix is of the order of n u, and the factor agrees with numpy.linalg.cholesky;
  * a leading minor that is not positive definite is reported with its order, the columns
    before it factored exactly.
"""
import numpy as np
import pytest

from oracle import oracle_cholesky_lower


def integer_factor(seed, n):
    g = np.random.default_rng(seed)
    L0 = np.tril(g.integers(-2, 3, size=(n, n)).astype(np.float64), -1)
    L0 += np.diag(g.choice([1.0, 2.0, 4.0], size=n))
    return L0


def with_nan_upper(A):
    A = np.asfortranarray(A.copy())
    A[np.triu_indices(A.shape[0], 1)] = np.nan
    return A


@pytest.mark.parametrize("n", [1, 2, 7, 64, 129, 300])
def test_integer_factor_recovered_exactly(n):
    L0 = integer_factor(n, n)
    A0 = L0 @ L0.T
    assert np.abs(A0).max() < 2 ** 40
    A = with_nan_upper(A0)
    assert oracle_cholesky_lower(A) == 0
    assert np.array_equal(np.tril(A), L0)
    assert np.isnan(A[np.triu_indices(n, 1)]).all()


def test_worked_example():
    A = np.asfortranarray(np.array([[4.0, 2.0], [2.0, 5.0]]))
    assert oracle_cholesky_lower(A) == 0
    assert np.array_equal(A, np.array([[2.0, 2.0], [1.0, 2.0]]))


def test_random_spd_backward_error_and_numpy():
    n = 400
    g = np.random.default_rng(21)
    X = g.uniform(-1, 1, size=(n, n))
    A0 = X @ X.T + n * np.eye(n)
    A = with_nan_upper(A0)
    assert oracle_cholesky_lower(A) == 0
    L = np.tril(A)
    assert np.linalg.norm(A0 - L @ L.T) / np.linalg.norm(A0) < 10 * n * 2.0 ** -53
    assert np.allclose(L, np.linalg.cholesky(A0), rtol=0, atol=1e-12 * np.abs(L).max())


@pytest.mark.parametrize("n,p", [(5, 0), (40, 17), (130, 129)])
def test_not_positive_definite_reported(n, p):
    L0 = integer_factor(100 + n, n)
    A0 = L0 @ L0.T
    A0[p, p] -= L0[p, p] ** 2 + 1.0   # the pivot of column p becomes -1
    A = with_nan_upper(A0)
    assert oracle_cholesky_lower(A) == p + 1
    assert np.array_equal(np.tril(A)[:, :p], L0[:, :p])

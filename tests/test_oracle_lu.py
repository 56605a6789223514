"""Pins of the oracle's LU factorization without pivoting (oracle_lu_nopiv).

  * A = L0 U0 with small-integer unit-lower L0 and upper U0: the factorization without pivoting
    is unique, and every intermediate of the elimination is an integer (each multiplier is an
    exact quotient), so the oracle must return L0 and U0 exactly;
  * reals: the backward error ||A - L U||_F / ||A||_F of a diagonally dominant matrix is of the
    order of n u, and L U reproduces A (numpy.matmul as the independent product);
  * a zero pivot is reported with its position.
"""
import numpy as np
import pytest

from oracle import oracle_lu_nopiv


def integer_factors(seed, n):
    g = np.random.default_rng(seed)
    L0 = np.tril(g.integers(-2, 3, size=(n, n)).astype(np.float64), -1) + np.eye(n)
    U0 = np.triu(g.integers(-2, 3, size=(n, n)).astype(np.float64), 1)
    U0 += np.diag(g.choice([1.0, 2.0, 4.0, -1.0, -2.0], size=n))
    return L0, U0


@pytest.mark.parametrize("n", [1, 2, 7, 64, 129, 300])
def test_integer_factors_recovered_exactly(n):
    L0, U0 = integer_factors(n, n)
    A = np.asfortranarray(L0 @ U0)
    assert np.abs(A).max() < 2 ** 40
    assert oracle_lu_nopiv(A) == 0
    assert np.array_equal(np.tril(A, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(A), U0)


def test_diagonally_dominant_backward_error():
    n = 400
    g = np.random.default_rng(9)
    A0 = g.uniform(-1, 1, size=(n, n)) + n * np.eye(n)
    A = np.asfortranarray(A0.copy())
    assert oracle_lu_nopiv(A) == 0
    L, U = np.tril(A, -1) + np.eye(n), np.triu(A)
    err = np.linalg.norm(L @ U - A0) / np.linalg.norm(A0)
    assert err < n * 2.0 ** -53


def test_zero_pivot_reported():
    A = np.asfortranarray(np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 1.0], [1.0, 1.0, 1.0]]))
    assert oracle_lu_nopiv(A) == 2   # after the first step the second pivot is 4 - 2*2 = 0

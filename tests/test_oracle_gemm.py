"""Pins for the CPU oracle's GEMM and recursive Strassen (CPU only).

Nothing here compares the oracle with a retyped copy of itself: the pins are
numpy.matmul on integer data (exact, so any correct method agrees bit for bit),
exact rational arithmetic (fractions) on tiny real inputs, closed forms
(identity and all-ones operands), the BLAS conventions for alpha/beta, and the
error bound of recursive summation.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, oracle_dgemm_dot2, oracle_strassen, fortran, rel_fro

U = 2.0 ** -53


def _int_problem(seed, m, n, k, ld_pad=0):
    g = np.random.default_rng(seed)
    A = W.integers(g, m, k, ld=m + ld_pad)
    B = W.integers(g, k, n, ld=k + ld_pad)
    C = W.integers(g, m, n, ld=m + ld_pad)
    return A, B, C


SMALL = [(m, n, k) for m in (1, 2, 3, 5, 8) for n in (1, 2, 4, 7) for k in (1, 2, 3, 6, 9)]


@pytest.mark.parametrize("m,n,k", SMALL)
def test_classical_integer_equals_numpy(m, n, k):
    A, B, C = _int_problem(m * 100 + n * 10 + k, m, n, k, ld_pad=(m + k) % 3)
    want = 3.0 * (np.asarray(A) @ np.asarray(B)) - 2.0 * np.asarray(C)
    got = oracle_dgemm(A, B, C.copy(order="F"), alpha=3.0, beta=-2.0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("m,n,k", SMALL + [(17, 33, 65), (64, 64, 64), (100, 31, 77), (129, 130, 131)])
def test_strassen_integer_equals_numpy(levels, m, n, k):
    A, B, C = _int_problem(7 + m + n + k, m, n, k, ld_pad=1)
    want = np.asarray(A) @ np.asarray(B) + np.asarray(C)
    got = oracle_strassen(A, B, C.copy(order="F"), alpha=1.0, beta=1.0, levels=levels)
    assert np.array_equal(got, want)


def test_closed_forms():
    m, n, k = 37, 21, 50
    g = np.random.default_rng(3)
    B = W.uniform(g, k, n)
    ones_a = fortran(np.ones((m, k)))
    ones_b = fortran(np.ones((k, n)))
    C = fortran(np.zeros((m, n)))
    # all-ones operands: every entry is exactly k
    for levels in (0, 1, 2):
        out = (oracle_dgemm(ones_a, ones_b, C.copy(order="F"), 1.0, 0.0) if levels == 0 else
               oracle_strassen(ones_a, ones_b, C.copy(order="F"), 1.0, 0.0, levels))
        assert np.all(out == k)
    # identity on the left returns B exactly, also through Strassen (I's quadrant
    # sums are 0/1/2 and products of a small integer with b are exact)
    I = fortran(np.eye(k))
    Ck = fortran(np.zeros((k, n)))
    assert np.array_equal(oracle_dgemm(I, B, Ck.copy(order="F"), 1.0, 0.0), np.asarray(B))


def test_beta_zero_does_not_read_c_and_alpha_zero_does_not_read_ab():
    m, n, k = 9, 7, 5
    g = np.random.default_rng(4)
    A, B = W.uniform(g, m, k), W.uniform(g, k, n)
    C = fortran(np.full((m, n), np.nan))
    for levels in (0, 1, 2):
        out = (oracle_dgemm(A, B, C.copy(order="F"), 1.0, 0.0) if levels == 0 else
               oracle_strassen(A, B, C.copy(order="F"), 1.0, 0.0, levels))
        assert np.all(np.isfinite(out))
    An = fortran(np.full((m, k), np.nan))
    C2 = W.uniform(g, m, n)
    out = oracle_dgemm(An, B, C2.copy(order="F"), 0.0, 2.0)
    assert np.array_equal(out, 2.0 * np.asarray(C2))
    out = oracle_strassen(An, B, C2.copy(order="F"), 0.0, 2.0, 2)
    assert np.array_equal(out, 2.0 * np.asarray(C2))


def _exact(A, B):
    A = [[Fraction(x) for x in row] for row in np.asarray(A).tolist()]
    B = [[Fraction(x) for x in row] for row in np.asarray(B).tolist()]
    m, k, n = len(A), len(B), len(B[0])
    return [[sum(A[i][p] * B[p][j] for p in range(k)) for j in range(n)] for i in range(m)], A, B


def test_classical_and_dot2_against_exact_rationals():
    g = np.random.default_rng(5)
    m, n, k = 6, 5, 40
    A, B = W.uniform(g, m, k), W.uniform(g, k, n)
    exact, Af, Bf = _exact(A, B)
    C = fortran(np.zeros((m, n)))
    plain = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 0.0)
    comp = oracle_dgemm_dot2(A, B, C.copy(order="F"), 1.0, 0.0)
    for i in range(m):
        for j in range(n):
            absdot = float(sum(abs(Af[i][p] * Bf[p][j]) for p in range(k)))
            # recursive summation: |err| <= gamma_k sum |a||b|  (Higham, Thm 3.1)
            gamma = k * U / (1 - k * U)
            assert abs(Fraction(plain[i, j]) - exact[i][j]) <= Fraction(gamma * absdot)
            # Dot2: |err| <= u|s| + gamma_k^2 sum|a||b| (Ogita-Rump-Oishi)
            assert abs(Fraction(comp[i, j]) - exact[i][j]) <= Fraction(
                U * abs(float(exact[i][j])) + 2 * gamma * gamma * absdot)


@pytest.mark.parametrize("levels", [1, 2])
def test_strassen_reals_close_to_exact(levels):
    g = np.random.default_rng(6 + levels)
    m, n, k = 40, 36, 44
    A, B, C = W.uniform(g, m, k), W.uniform(g, k, n), W.uniform(g, m, n)
    ref = oracle_dgemm_dot2(A, B, C.copy(order="F"), 1.0, 1.0)
    got = oracle_strassen(A, B, C.copy(order="F"), 1.0, 1.0, levels)
    assert rel_fro(got, ref) < 1e-14
    # a plain-definition result is closer or comparable
    cl = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    assert rel_fro(cl, ref) < 1e-15


def test_strassen_error_grows_but_stays_small_at_512():
    g = np.random.default_rng(11)
    n = 512
    A, B, C = W.uniform(g, n, n), W.uniform(g, n, n), W.uniform(g, n, n)
    ref = oracle_dgemm_dot2(A, B, C.copy(order="F"), 1.0, 1.0)
    errs = []
    for levels in (0, 1, 2):
        out = (oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0) if levels == 0 else
               oracle_strassen(A, B, C.copy(order="F"), 1.0, 1.0, levels))
        errs.append(rel_fro(out, ref))
    assert errs[0] < 1e-14 and errs[1] < 1e-13 and errs[2] < 1e-12
    assert errs[2] > errs[0]


def test_planted_oracle_mistake_is_caught():
    """A transposed operand (a plausible slip) is caught by the numpy pin."""
    A, B, C = _int_problem(1, 6, 6, 6)
    want = np.asarray(A) @ np.asarray(B)
    wrong = oracle_dgemm(fortran(np.asarray(A).T), B, fortran(np.zeros((6, 6))), 1.0, 0.0)
    assert not np.array_equal(wrong, want)

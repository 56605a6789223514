"""Pins of the oracle's Winograd variant (oracle_winograd, oracle.tables.WINOGRAD) against
things it does not compute itself: the matrix-multiplication tensor (the flattened table must
reproduce C = A*B exactly on symbols), numpy.matmul on small integers (exact at every level,
so any correct method agrees bit for bit), the closed forms, and the error of the plain
definition on reals."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, oracle_strassen, oracle_winograd, rel_fro
from oracle import tables as T


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_winograd_table_is_matrix_multiplication(levels):
    tab = T.winograd_table(levels)
    assert len(tab) == 7 ** levels
    assert np.array_equal(T.tensor_of(tab, levels), T.matmul_tensor(levels))


def test_winograd_table_counts_and_planted_sign():
    # operand terms 1+1+4+1+2+3+2 = 14 per side, C updates 4+1+1+1+2+3+2 = 14 (flattened)
    assert T.counts(T.winograd_table(1)) == (7, 14, 14, 14)
    bad = [list(map(list, row)) for row in T.WINOGRAD]
    bad[5][0][2] = ((0, 0), +1)                  # S2 = S1 + A00 instead of S1 - A00
    assert not np.array_equal(T.tensor_of(bad, 1), T.matmul_tensor(1))


SHAPES = [(1, 1, 1), (2, 2, 2), (3, 5, 7), (8, 8, 8), (17, 33, 65), (64, 64, 64), (100, 31, 77),
          (129, 130, 131)]


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_winograd_integer_equals_numpy(levels, m, n, k):
    g = np.random.default_rng(m * 7 + n * 3 + k + levels)
    A, B, C = W.integers(g, m, k, m + 1), W.integers(g, k, n, k + 2), W.integers(g, m, n)
    want = 2.0 * (np.asarray(A) @ np.asarray(B)) - np.asarray(C)
    got = oracle_winograd(A, B, C.copy(order="F"), 2.0, -1.0, levels)
    assert np.array_equal(got, want)


def test_winograd_beta_zero_and_levels_zero():
    A, B, C = W.problem(5, 40, 30, 20, "uniform")
    Cn = np.full_like(C, np.nan)
    assert np.array_equal(oracle_winograd(A, B, Cn.copy(order="F"), 1.0, 0.0, 0),
                          oracle_dgemm(A, B, np.zeros_like(C, order="F"), 1.0, 0.0))
    assert np.isfinite(oracle_winograd(A, B, Cn.copy(order="F"), 1.0, 0.0, 2)).all()


@pytest.mark.parametrize("levels", [1, 2])
def test_winograd_error_on_reals(levels):
    """Strassen-like error: close to the plain definition, the same order as Strassen's."""
    A, B, C = W.problem(6, 256, 256, 256, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    ew = rel_fro(oracle_winograd(A, B, C.copy(order="F"), 1.0, 1.0, levels), ref)
    es = rel_fro(oracle_strassen(A, B, C.copy(order="F"), 1.0, 1.0, levels), ref)
    assert ew < 1e-13
    assert ew < 20 * es

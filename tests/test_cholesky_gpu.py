"""Cholesky factorization with Strassen trailing updates (strassen_dpotrf_lower) on the GPU,
against the oracle's plain right-looking factorization (oracle/oracle_cholesky_lower):

  * A = L0 L0^T with a small-integer lower-triangular L0 (diagonal 1, 2 or 4): every step is
    exact (integer products and sums, Strassen included, divisions by powers of two, square
    roots of perfect squares), so the factor must be L0 bit for bit, for block widths that leave
    a ragged last block column and for 0 to 3 levels of Strassen in the updates; the strict upper
    triangle (NaN here) is never read or written;
  * reals: a random symmetric positive definite matrix, compared with the oracle's factor and by
    the backward error;
  * a leading minor that is not positive definite is reported with its order (info).
"""
import numpy as np
import pytest

from oracle import oracle_cholesky_lower, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu


def integer_factor(seed, n):
    g = np.random.default_rng(seed)
    L0 = np.tril(g.integers(-2, 3, size=(n, n)).astype(np.float64), -1)
    L0 += np.diag(g.choice([1.0, 2.0, 4.0], size=n))
    return L0


def nan_upper(A):
    A = np.asfortranarray(A.copy())
    A[np.triu_indices(A.shape[0], 1)] = np.nan
    return A


@pytest.mark.parametrize("n,nb,levels", [(64, 64, 0), (200, 64, 1), (1000, 256, 1),
                                         (2500, 1024, 2), (4400, 2048, 1), (4400, 2048, 3),
                                         (4400, 2048, -1)])
def test_integer_factor_exact(n, nb, levels):
    print(f"case cholesky integer n={n} nb={nb} L={levels}", flush=True)
    L0 = integer_factor(n, n)
    A = nan_upper(L0 @ L0.T)
    assert np.abs(A[np.tril_indices(n)]).max() < 2 ** 40
    dA = sx.to_device(A)
    info = sx.potrf_lower(dA, nb, levels)
    torch.cuda.synchronize()
    got = sx.to_host(dA)
    assert info == 0
    assert np.array_equal(np.tril(got), L0)
    assert np.isnan(got[np.triu_indices(n, 1)]).all()


@pytest.mark.parametrize("levels", [0, 1])
def test_random_spd_against_oracle(levels):
    n, nb = 3000, 1024
    print(f"case cholesky reals n={n} L={levels}", flush=True)
    g = np.random.default_rng(31)
    X = g.uniform(-1, 1, size=(n, n))
    A0 = X @ X.T + n * np.eye(n)
    dA = sx.to_device(nan_upper(A0))
    assert sx.potrf_lower(dA, nb, levels) == 0
    torch.cuda.synchronize()
    L = np.tril(sx.to_host(dA))
    ref = nan_upper(A0)
    assert oracle_cholesky_lower(ref) == 0
    assert rel_fro(L, np.tril(ref)) < 1e-12
    assert np.linalg.norm(A0 - L @ L.T) / np.linalg.norm(A0) < 1e-14


@pytest.mark.parametrize("n,p", [(300, 17), (2500, 1500), (2500, 2499)])
def test_not_positive_definite_reported(n, p):
    print(f"case cholesky not SPD n={n} p={p}", flush=True)
    L0 = integer_factor(7 + n, n)
    A0 = L0 @ L0.T
    A0[p, p] -= L0[p, p] ** 2 + 1.0
    dA = sx.to_device(nan_upper(A0))
    info = sx.potrf_lower(dA, 1024, 1)
    torch.cuda.synchronize()
    assert info == p + 1
    got = sx.to_host(dA)
    assert np.array_equal(np.tril(got)[:, :p], L0[:, :p])


def test_empty_and_errors():
    dA = torch.zeros((8, 8), dtype=torch.float64, device="cuda").t()   # column-major
    assert sx.potrf_lower(dA[:0, :0], 64, 0) == 0
    with pytest.raises(sx.StrassenError) as ei:
        sx.potrf_lower(dA, 48, 0)
    assert ei.value.code == -4

"""Three levels of Strassen (Sec. 3.5, eq. e:straprim4 with L = 3: 343 products) on the GPU, ABC.

  * small integers: every intermediate is exact (sums of up to eight entries of |x| <= 8, so
    |sum| <= 64, products <= 4096, partial sums far below 2^53): bit-exact against the oracle,
    in place and on block-padded copies (ragged sizes, odd leading dimensions, misalignment);
  * reals: relative Frobenius error <= 1e-10 against the plain-definition oracle (the tolerance
    of one and two levels, 1e-12 and 1e-11, continued by the same factor per level), and within
    a small factor of the oracle's own recursive three-level Strassen;
  * beta = 0 ignores NaN in C; 32768^3 (the size three levels are for) on sampled columns.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, oracle_strassen, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
TOL3 = 1e-10


def run(A, B, C, alpha, beta, lda=None, ldb=None, ldc=None, offset=0):
    dA = sx.to_device(A, ld=lda, offset=offset)
    dB = sx.to_device(B, ld=ldb, offset=offset)
    dC = sx.to_device(C, ld=ldc, offset=offset)
    sx.dgemm(dA, dB, dC, alpha, beta, 3, "abc")
    torch.cuda.synchronize()
    return sx.to_host(dC)


@pytest.mark.parametrize("shape", [(512, 512, 512), (1024, 1000, 1040), (301, 259, 271),
                                   (130, 70, 200), (2048, 2048, 2048)])
def test_integer_bit_exact(shape):
    m, n, k = shape
    print(f"case L=3 integer {shape}", flush=True)
    A, B, C = W.problem(111, m, n, k, "integer")
    assert np.array_equal(run(A, B, C, 1.0, 1.0), oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0))


@pytest.mark.parametrize("shape", [(2048, 2048, 2048), (1024, 1000, 1040)])
def test_integer_bit_exact_beta_zero(shape):
    """beta = 0: each C block's first update (in the launch that first reaches it) writes
    alpha*M without reading C, while the same launch adds to other blocks that earlier launches
    wrote, and later launches add to it."""
    m, n, k = shape
    print(f"case L=3 integer beta0 {shape}", flush=True)
    A, B, C = W.problem(113, m, n, k, "integer")
    C[:] = np.nan
    got = run(A, B, C, -1.0, 0.0)
    assert np.array_equal(got, oracle_dgemm(A, B, np.zeros_like(C, order="F"), -1.0, 0.0))


@pytest.mark.parametrize("case", [(512, 512, 512, 1, 3, 1, 0), (640, 640, 640, 0, 0, 0, 1)])
def test_integer_odd_ld_and_misaligned(case):
    m, n, k, ea, eb, ec, off = case
    print(f"case L=3 layout {case}", flush=True)
    A, B, C = W.problem(112, m, n, k, "integer")
    got = run(A, B, C, 2.0, -1.0, lda=m + ea, ldb=k + eb, ldc=m + ec, offset=off)
    assert np.array_equal(got, oracle_dgemm(A, B, C.copy(order="F"), 2.0, -1.0))


@pytest.mark.parametrize("shape", [(1024, 1024, 1024), (777, 1001, 555)])
def test_reals_tolerance_and_strassen_error(shape):
    m, n, k = shape
    print(f"case L=3 reals {shape}", flush=True)
    A, B, C = W.problem(113, m, n, k, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), -0.75, 1.25)
    got = run(A, B, C, -0.75, 1.25)
    e_gpu = rel_fro(got, ref)
    e_o3 = rel_fro(oracle_strassen(A, B, C.copy(order="F"), -0.75, 1.25, 3), ref)
    assert e_gpu <= TOL3, e_gpu
    assert e_gpu <= 10 * e_o3 + 1e-16, (e_gpu, e_o3)


def test_beta_zero_ignores_nan_and_determinism():
    m = n = k = 512
    print("case L=3 beta0", flush=True)
    A, B, _ = W.problem(114, m, n, k, "integer")
    Cn = np.full((m, n), np.nan, order="F")
    got = run(A, B, Cn, 1.0, 0.0)
    assert np.array_equal(got, oracle_dgemm(A, B, np.zeros((m, n), order="F"), 1.0, 0.0))
    Ar, Br, Cr = W.problem(115, m, n, k, "uniform")
    assert np.array_equal(run(Ar, Br, Cr, 1.0, 1.0), run(Ar, Br, Cr, 1.0, 1.0))


def test_full_size_32768_sampled_columns():
    n = 32768
    print(f"case L=3 full size {n}", flush=True)
    A = W.device_uniform(121, n, n)
    B = W.device_uniform(122, n, n)
    C0 = W.device_uniform(123, n, n)
    C = C0.clone()
    sx.dgemm(A, B, C, 1.0, 1.0, 3, "abc")
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(3).choice(n, size=4, replace=False))
    idx = torch.as_tensor(cols, device=C.device)
    got = C[:, idx].cpu().numpy()
    del C
    A_h = sx.to_host(A)
    Bc = np.asfortranarray(B[:, idx].cpu().numpy())
    Cc = np.asfortranarray(C0[:, idx].cpu().numpy())
    ref = oracle_dgemm(A_h, Bc, Cc, 1.0, 1.0)
    assert rel_fro(got, ref) <= TOL3

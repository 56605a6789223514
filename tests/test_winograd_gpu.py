"""Winograd's variant (ABC, one and two levels) on the GPU against the CPU oracle.

  * small integers: exact (sums of at most four entries of |x| <= 8 per level), so bit-exact
    against the plain-definition oracle, in place and on block-padded copies;
  * reals: relative Frobenius error within the tolerances of Strassen at the same level (1e-12,
    1e-11) and within a small factor of the oracle's recursive Winograd variant (whose C-side
    sums associate differently: U2 = M1 + M6 is shared, the GPU adds each product in order);
  * 16384^3 at two levels on sampled columns.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, oracle_winograd, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
TOL = {1: 1e-12, 2: 1e-11}


def run(A, B, C, alpha, beta, levels, lda=None, ldb=None, ldc=None, offset=0):
    dA = sx.to_device(A, ld=lda, offset=offset)
    dB = sx.to_device(B, ld=ldb, offset=offset)
    dC = sx.to_device(C, ld=ldc, offset=offset)
    sx.dgemm_winograd(dA, dB, dC, alpha, beta, levels)
    torch.cuda.synchronize()
    return sx.to_host(dC)


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("shape", [(512, 512, 512), (1024, 1000, 1040), (300, 260, 270),
                                   (130, 70, 200), (2048, 2048, 2048)])
def test_integer_bit_exact(levels, shape):
    m, n, k = shape
    print(f"case winograd integer {shape} L={levels}", flush=True)
    A, B, C = W.problem(131, m, n, k, "integer")
    assert np.array_equal(run(A, B, C, 1.0, 1.0, levels),
                          oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0))


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("case", [(512, 512, 512, 1, 3, 1, 0), (640, 648, 640, 0, 0, 0, 1)])
def test_integer_odd_ld_and_misaligned(levels, case):
    m, n, k, ea, eb, ec, off = case
    print(f"case winograd layout {case} L={levels}", flush=True)
    A, B, C = W.problem(132, m, n, k, "integer")
    got = run(A, B, C, -1.0, 2.0, levels, lda=m + ea, ldb=k + eb, ldc=m + ec, offset=off)
    assert np.array_equal(got, oracle_dgemm(A, B, C.copy(order="F"), -1.0, 2.0))


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("shape", [(1024, 1024, 1024), (777, 1001, 555)])
def test_reals_tolerance(levels, shape):
    m, n, k = shape
    print(f"case winograd reals {shape} L={levels}", flush=True)
    A, B, C = W.problem(133, m, n, k, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 0.5, 1.5)
    e_gpu = rel_fro(run(A, B, C, 0.5, 1.5, levels), ref)
    e_o = rel_fro(oracle_winograd(A, B, C.copy(order="F"), 0.5, 1.5, levels), ref)
    assert e_gpu <= TOL[levels], e_gpu
    assert e_gpu <= 10 * e_o + 1e-16, (e_gpu, e_o)


def test_beta_zero_ignores_nan():
    m = n = k = 512
    print("case winograd beta0", flush=True)
    A, B, _ = W.problem(134, m, n, k, "integer")
    for levels in (1, 2):
        got = run(A, B, np.full((m, n), np.nan, order="F"), 1.0, 0.0, levels)
        assert np.array_equal(got, oracle_dgemm(A, B, np.zeros((m, n), order="F"), 1.0, 0.0))


def test_full_size_two_levels_sampled_columns():
    n = 16384
    print(f"case winograd full size {n}", flush=True)
    A, B, C0 = (W.device_uniform(s, n, n) for s in (141, 142, 143))
    C = C0.clone()
    sx.dgemm_winograd(A, B, C, 1.0, 1.0, 2)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(4).choice(n, size=8, replace=False))
    idx = torch.as_tensor(cols, device=C.device)
    ref = oracle_dgemm(sx.to_host(A), np.asfortranarray(B[:, idx].cpu().numpy()),
                       np.asfortranarray(C0[:, idx].cpu().numpy()), 1.0, 1.0)
    assert rel_fro(C[:, idx].cpu().numpy(), ref) <= TOL[2]


@pytest.mark.parametrize("shape,beta", [((8192, 8192, 8192), 1.0), ((8188, 8190, 8196), 0.0)])
def test_one_level_on_the_classical_kernel(shape, beta):
    """Where one-level ABC runs on the classical kernel, so does Winograd's variant: its chain
    sums S1..S4 / T1..T4 staged (two passes), seven classical launches adding each product to
    every C quadrant it reaches (M1 all four).  A workspace cap below the eight slots gives the
    all-products kernel: the same bits.  Sampled columns against the oracle (beta = 0: C, full
    of NaN, is not read); integers exact."""
    m, n, k = shape
    print(f"case winograd one level classical {shape} beta={beta}", flush=True)
    r32 = lambda x: -(-x // 32) * 32
    slots = 8 * (4 * r32((m // 2) * (k // 2)) + 4 * r32((k // 2) * (n // 2)))
    assert sx.workspace_size_winograd(m, n, k, 1) == slots
    cols = np.array([0, 5, n // 2 - 1, n // 2, n - 1])
    for kind in ("uniform", "integer"):
        A, B, C = W.problem(41, m, n, k, kind)
        if beta == 0.0:
            C[:] = np.nan
        dA, dB = sx.to_device(A), sx.to_device(B)

        def counted():
            for kk in sx.KERNEL_KINDS:
                sx.timing_collect(kk)
            sx.timing_enable(True)
            try:
                dC = sx.to_device(C)
                sx.dgemm_winograd(dA, dB, dC, 1.0, beta, 1)
                torch.cuda.synchronize()
            finally:
                sx.timing_enable(False)
            return (sx.to_host(dC), sx.timing_collect("outer_sums")[1],
                    sx.timing_collect("classical")[1], sx.timing_collect("all_products")[1])

        staged, *counts = counted()
        assert tuple(counts) == (2, 7, 0)
        try:
            sx.set_workspace_limit(slots // 2)
            fused, *counts = counted()
            assert tuple(counts) == (0, 0, 1)
        finally:
            sx.set_workspace_limit(0)
        assert np.array_equal(staged, fused)
        Cc = np.asfortranarray(C[:, cols]) if beta != 0.0 else np.zeros((m, len(cols)), order="F")
        ref = oracle_dgemm(A, np.asfortranarray(B[:, cols]), Cc, 1.0, beta)
        if kind == "integer":
            assert np.array_equal(staged[:, cols], ref)
        else:
            assert rel_fro(staged[:, cols], ref) <= TOL[1]

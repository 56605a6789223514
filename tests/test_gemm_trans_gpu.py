"""strassen_gemm (transposed operands, Sec. 2.2) and the drop-in BLAS library (dgemm_,
cblas_dgemm) on the GPU, against the oracle on op(A), op(B):
  * small integers: bit-exact for every transpose pair, level and variant;
  * reals: bitwise equal to strassen_dgemm on the explicitly transposed matrices (the packed
    copy changes no operation), and within the Strassen tolerance of the oracle;
  * dgemm_ / cblas_dgemm with host (numpy) and device (torch) operands."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
BLAS = os.path.join(os.path.dirname(sx.LIB_PATH), "libstrassen_blas.so")
PAIRS = [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")]


def stored(X, t):
    """The matrix the caller stores for op(X) = X ('N') or X^T ('T')."""
    return np.asfortranarray(X.T) if t == "T" else X


@pytest.mark.parametrize("ta,tb", PAIRS)
@pytest.mark.parametrize("levels,variant", [(0, "abc"), (1, "abc"), (1, "ab"), (1, "naive"),
                                            (2, "abc"), (2, "ab"), (2, "naive")])
def test_gemm_transposes_integer_exact(ta, tb, levels, variant):
    m, n, k = 301, 259, 270
    print(f"case gemm {ta}{tb} L={levels} {variant}", flush=True)
    A, B, C = W.problem(101, m, n, k, "integer")
    want = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    dC = sx.to_device(C)
    sx.gemm(sx.to_device(stored(A, ta)), sx.to_device(stored(B, tb)), dC, 1.0, 1.0, ta, tb,
            levels, variant)
    torch.cuda.synchronize()
    assert np.array_equal(sx.to_host(dC), want)


@pytest.mark.parametrize("ta,tb", PAIRS)
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_gemm_transposes_bitwise_with_dgemm(ta, tb, levels):
    m, n, k = 1030, 770, 902
    print(f"case gemm bitwise {ta}{tb} L={levels}", flush=True)
    A, B, C = W.problem(102, m, n, k, "uniform")
    dC = sx.to_device(C)
    sx.gemm(sx.to_device(stored(A, ta)), sx.to_device(stored(B, tb)), dC, -0.5, 1.5, ta, tb,
            levels, "abc")
    ref_c = sx.to_device(C)
    sx.dgemm(sx.to_device(A), sx.to_device(B), ref_c, -0.5, 1.5, levels, "abc")
    torch.cuda.synchronize()
    got = sx.to_host(dC)
    assert np.array_equal(got, sx.to_host(ref_c))
    err = rel_fro(got, oracle_dgemm(A, B, C.copy(order="F"), -0.5, 1.5))
    assert err <= (1e-11 if levels == 2 else 1e-12)


@pytest.mark.parametrize("m,n,k,ldb_extra,shift", [(64, 64, 64, 0, 0), (130, 66, 17, 0, 0),
                                                   (255, 129, 300, 1, 0), (1, 1, 1, 0, 0),
                                                   (512, 300, 1000, 0, 1), (700, 1000, 64, 3, 1)])
def test_transposed_b_read_in_place_by_the_tile_kernel(m, n, k, ldb_extra, shift):
    # classical products too small for the classical kernel read op(B) = B^T in place on the
    # tile kernel (16-byte pairs where n, ldb and B's alignment allow, else element by element,
    # shift = 1: B one element past a 16-byte boundary); the same bits as the product on an
    # explicit transposed copy, exact on integers
    print(f"case gemm NT in place {m}x{n}x{k} ldb+{ldb_extra} shift {shift}", flush=True)
    for kind in ("integer", "uniform"):
        A, B, C = W.problem(103, m, n, k, kind)
        Bt = np.asfortranarray(B.T)
        buf = torch.zeros(((n + ldb_extra) * k + 2,), dtype=torch.float64, device="cuda")
        dBt = buf[shift:shift + (n + ldb_extra) * k].view(k, n + ldb_extra).t()[:n, :]
        dBt.copy_(torch.as_tensor(Bt, device="cuda"))
        dC = sx.to_device(C)
        sx.gemm(sx.to_device(A), dBt, dC, 0.75, -1.25, "N", "T", 0, "abc")
        ref_c = sx.to_device(C)
        sx.dgemm(sx.to_device(A), sx.to_device(B), ref_c, 0.75, -1.25, 0, "abc")
        torch.cuda.synchronize()
        got = sx.to_host(dC)
        assert np.array_equal(got, sx.to_host(ref_c))
        if kind == "integer":
            assert np.array_equal(got, oracle_dgemm(A, B, C.copy(order="F"), 0.75, -1.25))


def test_gemm_member_chosen_by_library():
    m, n, k = 2048, 2048, 2048
    print("case gemm levels=-1", flush=True)
    A, B, C = W.problem(103, m, n, k, "uniform")
    dC = sx.to_device(C)
    sx.gemm(sx.to_device(stored(A, "T")), sx.to_device(B), dC, 1.0, 1.0, "T", "N", -1)
    torch.cuda.synchronize()
    assert rel_fro(sx.to_host(dC), oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)) <= 1e-11


def _blas():
    L = ctypes.CDLL(BLAS)
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
    dbl = ctypes.POINTER(ctypes.c_double)
    L.dgemm_.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ip, ip, ip, dbl, dp, ip, dp, ip, dbl, dp, ip]
    L.dgemm_.restype = None
    ci = ctypes.c_int
    L.cblas_dgemm.argtypes = [ci, ci, ci, ci, ci, ci, ctypes.c_double, dp, ci, dp, ci,
                              ctypes.c_double, dp, ci]
    L.cblas_dgemm.restype = None
    return L


def _dgemm_(L, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    i = lambda v: ctypes.byref(ctypes.c_int(v))
    d = lambda v: ctypes.byref(ctypes.c_double(v))
    L.dgemm_(ta.encode(), tb.encode(), i(m), i(n), i(k), d(alpha), A, i(lda), B, i(ldb), d(beta),
             C, i(ldc))


@pytest.mark.parametrize("ta,tb", PAIRS)
def test_dgemm_host_operands(ta, tb):
    m, n, k = 700, 650, 610
    print(f"case dgemm_ host {ta}{tb}", flush=True)
    A, B, C = W.problem(104, m, n, k, "integer")
    As, Bs = stored(A, ta), stored(B, tb)
    Cg = C.copy(order="F")
    _dgemm_(_blas(), ta, tb, m, n, k, 1.0, As.ctypes.data, As.shape[0], Bs.ctypes.data,
            Bs.shape[0], 1.0, Cg.ctypes.data, m)
    assert np.array_equal(Cg, oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0))


def test_dgemm_device_operands_and_leading_dimensions():
    m, n, k = 1100, 900, 1000
    print("case dgemm_ device", flush=True)
    A, B, C = W.problem(105, m, n, k, "uniform")
    dA, dB, dC = sx.to_device(A, ld=m + 6), sx.to_device(stored(B, "T"), ld=n + 2), sx.to_device(C, ld=m + 4)
    _dgemm_(_blas(), "N", "T", m, n, k, 2.0, dA.data_ptr(), m + 6, dB.data_ptr(), n + 2, -1.0,
            dC.data_ptr(), m + 4)
    got = sx.to_host(dC)
    assert rel_fro(got, oracle_dgemm(A, B, C.copy(order="F"), 2.0, -1.0)) <= 1e-11


def test_cblas_row_major_host():
    m, n, k = 333, 444, 555
    print("case cblas row-major", flush=True)
    A, B, C = W.problem(106, m, n, k, "integer")
    Ar, Br, Cr = np.ascontiguousarray(A), np.ascontiguousarray(B), np.ascontiguousarray(C)
    _blas().cblas_dgemm(101, 111, 111, m, n, k, 1.0, Ar.ctypes.data, k, Br.ctypes.data, n, 1.0,
                        Cr.ctypes.data, n)
    assert np.array_equal(Cr, oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0))

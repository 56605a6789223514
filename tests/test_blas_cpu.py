"""Host-side checks of strassen_gemm (transposed operands) and the drop-in BLAS library
libstrassen_blas.so (dgemm_, cblas_dgemm): argument errors are reported before any device call,
with BLAS's parameter numbers, and leave C untouched."""
import ctypes
import os

import numpy as np
import pytest

import paper_1605_01078_amd as sx

BLAS = os.path.join(os.path.dirname(sx.LIB_PATH), "libstrassen_blas.so")


def blas():
    L = ctypes.CDLL(BLAS)
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
    L.dgemm_.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ip, ip, ip, ctypes.POINTER(ctypes.c_double),
                         dp, ip, dp, ip, ctypes.POINTER(ctypes.c_double), dp, ip]
    L.dgemm_.restype = None
    return L


def call_dgemm_(L, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    i = lambda v: ctypes.byref(ctypes.c_int(v))
    d = lambda v: ctypes.byref(ctypes.c_double(v))
    L.dgemm_(ta, tb, i(m), i(n), i(k), d(alpha), A, i(lda), B, i(ldb), d(beta), C, i(ldc))


def test_blas_library_exports():
    L = ctypes.CDLL(BLAS)
    assert hasattr(L, "dgemm_") and hasattr(L, "cblas_dgemm")


@pytest.mark.parametrize("args,info", [
    ((b"X", b"N", 4, 4, 4, 4, 4, 4), 1),
    ((b"N", b"Q", 4, 4, 4, 4, 4, 4), 2),
    ((b"N", b"N", -1, 4, 4, 4, 4, 4), 3),
    ((b"N", b"N", 4, -1, 4, 4, 4, 4), 4),
    ((b"N", b"N", 4, 4, -1, 4, 4, 4), 5),
    ((b"N", b"N", 4, 4, 4, 3, 4, 4), 8),
    ((b"T", b"N", 4, 4, 6, 5, 6, 4), 8),      # A is k x m when transposed: lda >= k
    ((b"N", b"N", 4, 4, 6, 4, 5, 4), 10),
    ((b"N", b"T", 4, 7, 4, 4, 6, 4), 10),     # B is n x k when transposed: ldb >= n
    ((b"N", b"N", 4, 4, 4, 4, 4, 3), 13),
])
def test_dgemm_illegal_arguments(args, info, capfd):
    ta, tb, m, n, k, lda, ldb, ldc = args
    C = np.full((8, 8), 7.0, order="F")
    A = np.zeros((8, 8), order="F")
    call_dgemm_(blas(), ta, tb, m, n, k, 1.0, A.ctypes.data, lda, A.ctypes.data, ldb, 1.0,
                C.ctypes.data, ldc)
    err = capfd.readouterr().err
    assert f"parameter number {info:2d} had an illegal value" in err
    assert (C == 7.0).all()


def test_dgemm_quick_return_without_device():
    C = np.full((4, 4), 3.0, order="F")
    call_dgemm_(blas(), b"N", b"N", 0, 4, 4, 1.0, None, 1, None, 4, 1.0, C.ctypes.data, 1)
    call_dgemm_(blas(), b"N", b"N", 4, 4, 4, 0.0, None, 4, None, 4, 1.0, C.ctypes.data, 4)
    assert (C == 3.0).all()


@pytest.mark.parametrize("args,code", [
    ((b"X", b"N", 4, 4, 4, 4, 4, 4, 1, 0), -1),
    ((b"N", b"?", 4, 4, 4, 4, 4, 4, 1, 0), -2),
    ((b"N", b"N", -1, 4, 4, 4, 4, 4, 1, 0), -3),
    ((b"T", b"N", 4, 4, 6, 5, 6, 4, 1, 0), -8),
    ((b"N", b"T", 4, 7, 4, 4, 6, 4, 1, 0), -10),
    ((b"N", b"N", 4, 4, 4, 4, 4, 3, 1, 0), -13),
    ((b"N", b"N", 4, 4, 4, 4, 4, 4, 4, 0), -14),
    ((b"N", b"N", 4, 4, 4, 4, 4, 4, 3, 1), -15),
    ((b"N", b"N", 4, 4, 4, 4, 4, 4, -2, 0), -14),
    ((b"N", b"N", 4, 4, 4, 4, 4, 4, 1, 5), -15),
])
def test_strassen_gemm_argument_codes(args, code):
    ta, tb, m, n, k, lda, ldb, ldc, lev, var = args
    fake = 1 << 20   # never dereferenced: the checks fail first
    rc = sx.lib().strassen_gemm(ta, tb, m, n, k, 1.0, fake, lda, fake, ldb, 1.0, fake, ldc, lev,
                                var, None)
    assert rc == code, sx.last_error()

"""CPU oracle for one- and two-level Strassen C := alpha*A*B + beta*C.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the HIP library
(no kernels, headers, tables or helpers); both sides only share the seeded
input generators in ``workloads``.

Contents
  oracle_dgemm(A, B, C, alpha, beta)        plain definition (Sec. 2.1/2.2)
  oracle_strassen(A, B, C, alpha, beta, L)  recursive textbook Strassen (Sec. 3.1-3.2)
  oracle_winograd(A, B, C, alpha, beta, L)  recursive Winograd variant (Strassen-like scheme)
  oracle_lu_nopiv(A)                        LU without pivoting, plain elimination
  oracle_cholesky_lower(A)                  Cholesky A = L L^T, plain right-looking
  oracle_dgemm_dot2(...)                    compensated reference (error yardstick)
  tables                                    the paper's operation tables (Fig. one-level,
                                            Fig. two-level via the Kronecker rule)
  tiny                                      pure-Python loops for tiny sizes
  costmodel                                 the paper's performance model (Sec. 4.2)
  mlp                                       fp64 numpy MLP (selector gradients)
  lowprec                                   bf16 rounding / hi-lo split and the
                                            reduced-precision Strassen oracle

Matrices are numpy float64 arrays in Fortran (column-major) order; a view
``X[:rows, :cols]`` of a larger Fortran array carries its leading dimension.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, dbl, ptr = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        sig = [i64, i64, i64, dbl, ptr, i64, ptr, i64, dbl, ptr, i64]
        lib.oracle_dgemm.argtypes = sig
        lib.oracle_dgemm.restype = ctypes.c_int
        lib.oracle_dgemm_dot2.argtypes = sig
        lib.oracle_dgemm_dot2.restype = ctypes.c_int
        lib.oracle_strassen.argtypes = sig + [ctypes.c_int]
        lib.oracle_strassen.restype = ctypes.c_int
        lib.oracle_winograd.argtypes = sig + [ctypes.c_int]
        lib.oracle_winograd.restype = ctypes.c_int
        lib.oracle_lu_nopiv.argtypes = [i64, ptr, i64]
        lib.oracle_lu_nopiv.restype = ctypes.c_int
        lib.oracle_cholesky_lower.argtypes = [i64, ptr, i64]
        lib.oracle_cholesky_lower.restype = ctypes.c_int
        _lib = lib
    return _lib


def _colmajor(X, name):
    """Pointer and leading dimension of a float64 column-major matrix view."""
    if X.dtype != np.float64 or X.ndim != 2:
        raise TypeError(f"{name}: expected a 2-D float64 array")
    if X.shape[0] > 1 and X.strides[0] != 8:
        raise ValueError(f"{name}: rows must be contiguous (column-major)")
    ld = X.strides[1] // 8 if X.shape[1] > 1 else max(1, X.shape[0])
    return X.ctypes.data, max(ld, max(1, X.shape[0]))


def _call(fn, A, B, C, alpha, beta, *extra):
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or C.shape != (m, n):
        raise ValueError("shape mismatch")
    pa, lda = _colmajor(A, "A")
    pb, ldb = _colmajor(B, "B")
    pc, ldc = _colmajor(C, "C")
    rc = fn(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc, *extra)
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")
    return C


def oracle_dgemm(A, B, C, alpha=1.0, beta=1.0):
    """C := alpha*A*B + beta*C in place (plain definition, sequential sum over p)."""
    return _call(_load().oracle_dgemm, A, B, C, alpha, beta)


def oracle_dgemm_dot2(A, B, C, alpha=1.0, beta=1.0):
    """Same as oracle_dgemm with each dot product in doubled working precision."""
    return _call(_load().oracle_dgemm_dot2, A, B, C, alpha, beta)


def oracle_strassen(A, B, C, alpha=1.0, beta=1.0, levels=1):
    """C := alpha*(A*B by `levels` levels of recursive Strassen) + beta*C in place."""
    return _call(_load().oracle_strassen, A, B, C, alpha, beta, int(levels))


def oracle_winograd(A, B, C, alpha=1.0, beta=1.0, levels=1):
    """C := alpha*(A*B by `levels` levels of Winograd's variant) + beta*C in place."""
    return _call(_load().oracle_winograd, A, B, C, alpha, beta, int(levels))


def oracle_lu_nopiv(A):
    """A = L U in place (no pivoting); returns 0, or p + 1 if pivot p was exactly zero."""
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    pa, lda = _colmajor(A, "A")
    return _load().oracle_lu_nopiv(n, pa, lda)


def oracle_cholesky_lower(A):
    """A = L L^T in place, L in the lower triangle (the strict upper triangle is neither read
    nor written); returns 0, or p + 1 if the pivot of column p was not positive."""
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    pa, lda = _colmajor(A, "A")
    return _load().oracle_cholesky_lower(n, pa, lda)


def fortran(X, ld=None):
    """Copy X into a column-major array whose leading dimension is `ld`."""
    X = np.asarray(X, dtype=np.float64)
    rows, cols = X.shape
    ld = rows if ld is None else ld
    buf = np.zeros((max(ld, 1), cols), dtype=np.float64, order="F")
    buf[:rows, :] = X
    return buf[:rows, :]


def rel_fro(X, R):
    """Relative Frobenius distance ||X - R||_F / ||R||_F."""
    d = np.linalg.norm(np.asarray(X) - np.asarray(R))
    r = np.linalg.norm(np.asarray(R))
    return d / r if r > 0 else d

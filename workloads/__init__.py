"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers
and shapes.  Every matrix is returned as a float64 numpy array in Fortran
(column-major) order, optionally embedded in a buffer with a larger leading
dimension (the view keeps that leading dimension in its strides).

Workloads (shapes and distributions of the paper's experiments, Sec. 5):
  square      m = n = k, entries uniform on [-1, 1]
  rank-k      m = n = 16384 with k in {256, ..., 8192} (the SUMMA local update shape)
  integer     entries uniform on the integers -8..8 (small enough that every
              intermediate of one- and two-level Strassen is exact in FP64)
  wide-range  uniform[-1,1] entries with row i scaled by 2^u_i, u_i ~ U[-8, 8]
  batched     512 problems, m, n, k multiples of 64 in [256, 4096]
  selector    shapes log-uniform in [256, 20000]
"""
import numpy as np

SQUARE_SIZES = tuple(range(2048, 16384 + 1, 2048))
RANK_K_M = 16384
RANK_K_KS = (256, 512, 1024, 2048, 4096, 8192)


def rng(seed=0):
    return np.random.default_rng(seed)


def _embed(X, ld):
    rows, cols = X.shape
    ld = rows if ld is None else int(ld)
    if ld < max(1, rows):
        raise ValueError("leading dimension smaller than the row count")
    buf = np.zeros((max(ld, 1), cols), dtype=np.float64, order="F")
    buf[:rows, :] = X
    return buf[:rows, :]


def uniform(g, rows, cols, ld=None, lo=-1.0, hi=1.0):
    """rows x cols, i.i.d. uniform on [lo, hi)."""
    return _embed(g.uniform(lo, hi, size=(rows, cols)), ld)


def integers(g, rows, cols, ld=None, lo=-8, hi=8):
    """rows x cols, i.i.d. uniform on the integers lo..hi inclusive."""
    return _embed(g.integers(lo, hi + 1, size=(rows, cols)).astype(np.float64), ld)


def row_scale_exponents(g, rows, lo=-8.0, hi=8.0):
    return g.uniform(lo, hi, size=rows)


def wide_range(g, rows, cols, ld=None, scale_rows=True):
    """uniform[-1,1] entries; row i multiplied by 2^u_i with u_i ~ U[-8, 8]."""
    X = g.uniform(-1.0, 1.0, size=(rows, cols))
    if scale_rows:
        X = X * np.exp2(row_scale_exponents(g, rows))[:, None]
    return _embed(X, ld)


def problem(seed, m, n, k, kind="uniform", lda=None, ldb=None, ldc=None, c_zero=False):
    """(A, B, C) for one GEMM C := alpha*A*B + beta*C."""
    g = rng(seed)
    if kind == "uniform":
        A, B = uniform(g, m, k, lda), uniform(g, k, n, ldb)
        C = uniform(g, m, n, ldc)
    elif kind == "integer":
        A, B = integers(g, m, k, lda), integers(g, k, n, ldb)
        C = integers(g, m, n, ldc)
    elif kind == "wide_a":
        A, B = wide_range(g, m, k, lda), uniform(g, k, n, ldb)
        C = uniform(g, m, n, ldc)
    elif kind == "wide_b":
        A, B = uniform(g, m, k, lda), wide_range(g, k, n, ldb)
        C = uniform(g, m, n, ldc)
    elif kind == "wide_both":
        A, B = wide_range(g, m, k, lda), wide_range(g, k, n, ldb)
        C = uniform(g, m, n, ldc)
    else:
        raise ValueError(kind)
    if c_zero:
        C[...] = 0.0
    return A, B, C


def batched_shapes(seed=0, count=512, lo=256, hi=4096, step=64):
    """`count` (m, n, k) triples, each dimension uniform over the multiples of
    `step` in [lo, hi]."""
    g = rng(seed)
    vals = np.arange(lo, hi + 1, step)
    return [tuple(int(v) for v in g.choice(vals, size=3)) for _ in range(count)]


def selector_shapes(seed=0, count=20000, lo=256, hi=20000):
    """`count` (m, n, k) triples, each dimension log-uniform in [lo, hi], rounded."""
    g = rng(seed)
    x = np.exp(g.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    x = np.clip(np.rint(x), lo, hi).astype(np.int64)
    return [tuple(int(v) for v in row) for row in x]


def device_uniform(seed, rows, cols, ld=None, device="cuda", lo=-1.0, hi=1.0):
    """rows x cols column-major float64 torch tensor, i.i.d. uniform on [lo, hi), drawn on the
    device from a seeded torch generator (for sizes too large to draw on the host quickly)."""
    import torch
    ld = rows if ld is None else int(ld)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    buf = torch.empty((cols, max(ld, 1)), dtype=torch.float64, device=device)
    buf.uniform_(lo, hi, generator=g)
    return buf.t()[:rows, :]

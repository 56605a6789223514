"""Python binding of libstrassen.so: one- and two-level Strassen GEMM on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
The library must have been built (``python -m paper_1605_01078_amd.build``); importing the
functions below fails loudly if it is missing.  PyTorch supplies device memory and streams.

Matrices are column-major.  A column-major m x k matrix with leading dimension ld is a torch
tensor of shape (m, k) with strides (1, ld), e.g. ``torch.empty(k, ld).t()[:m]``;
:func:`colmajor` and :func:`to_device` build such tensors.
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstrassen.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "strassen.h")

ABC, AB, NAIVE = 0, 1, 2
VARIANTS = {"abc": ABC, "ab": AB, "naive": NAIVE}
COMPUTE = {"f64": 0, "bf16": 1, "bf16x3": 2}
PREC = {"f32": 0, "f64": 1}

_lib = None


class StrassenError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"strassen error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library (ctypes.CDLL); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1605_01078_amd.build`")
        # torch first: it loads its own HIP runtime under the same soname as the one the library
        # links, and a process must use one runtime (the library then binds to torch's; loaded
        # the other way round, torch's device calls can find no device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        i64, dbl, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        gemm = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, ci, ci]
        L.strassen_dgemm.argtypes = gemm + [vp]
        L.strassen_dgemm.restype = ci
        L.strassen_gemm.argtypes = [ctypes.c_char, ctypes.c_char] + gemm + [vp]
        L.strassen_gemm.restype = ci
        L.strassen_dgemm_winograd.argtypes = gemm[:-1] + [vp]
        L.strassen_dgemm_winograd.restype = ci
        L.strassen_workspace_size_winograd.argtypes = [i64, i64, i64, ci,
                                                       ctypes.POINTER(ctypes.c_size_t)]
        L.strassen_workspace_size_winograd.restype = ci
        L.strassen_dgetrf_nopiv.argtypes = [i64, vp, i64, i64, ci, vp]
        L.strassen_dgetrf_nopiv.restype = ci
        L.strassen_dpotrf_lower.argtypes = [i64, vp, i64, i64, ci, ctypes.POINTER(i64), vp]
        L.strassen_dpotrf_lower.restype = ci
        L.strassen_dgemm_noalloc.argtypes = gemm + [vp]
        L.strassen_dgemm_noalloc.restype = ci
        L.strassen_gemm_ex.argtypes = gemm + [ci, ci, ci, vp]
        L.strassen_gemm_ex.restype = ci
        L.strassen_workspace_size.argtypes = [i64, i64, i64, ci, ci, ctypes.POINTER(ctypes.c_size_t)]
        L.strassen_workspace_size.restype = ci
        L.strassen_workspace_size_ex.argtypes = [i64, i64, i64, ci, ci, ctypes.POINTER(ctypes.c_size_t)]
        L.strassen_workspace_size_ex.restype = ci
        L.strassen_set_workspace.argtypes = [vp, ctypes.c_size_t]
        L.strassen_set_workspace.restype = ci
        L.strassen_set_workspace_limit.argtypes = [ctypes.c_size_t]
        L.strassen_set_workspace_limit.restype = ci
        L.strassen_release_workspace.argtypes = []
        L.strassen_release_workspace.restype = ci
        L.strassen_table_size.argtypes = [ci]
        L.strassen_table_size.restype = ci
        ip = ctypes.POINTER(ci)
        L.strassen_table_get.argtypes = [ci, ci, ip, ip, ip, ip, ip, ip]
        L.strassen_table_get.restype = ci
        L.strassen_last_error.argtypes = []
        L.strassen_last_error.restype = ctypes.c_char_p
        L.strassen_set_tile_config.argtypes = [ci]
        L.strassen_set_tile_config.restype = ci
        L.strassen_version.argtypes = []
        L.strassen_version.restype = ctypes.c_char_p
        _optional(L)
        _lib = L
    return _lib


def _optional(L):
    """Signatures of the batched-mode and selector entry points."""
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp, ci, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    ops = [vp, ctypes.POINTER(vp), i64p, ctypes.POINTER(vp), i64p, ctypes.POINTER(vp), i64p,
           dbl, dbl, vp]
    specs = {
        "strassen_batched_plan": ([ci, i64p, i64p, i64p, ctypes.POINTER(ci), ctypes.POINTER(ci),
                                   ctypes.POINTER(vp)], ci),
        "strassen_batched_autotune": ([vp, ci, ctypes.c_uint64, vp], ci),
        "strassen_batched_choice": ([vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "strassen_batched_run": (ops, ci),
        "strassen_batched_capture": (ops, ci),
        "strassen_batched_replay": ([vp, vp], ci),
        "strassen_batched_destroy": ([vp], ci),
        "strassen_select": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ci,
                             ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "strassen_cost_model": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ci,
                                 ctypes.POINTER(ctypes.c_double)], ci),
        "strassen_selector_load": ([vp], ci),
        "strassen_selector_features": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ci,
                                        ctypes.POINTER(ctypes.c_float)], ci),
        "strassen_mlp_forward": ([vp, vp, ci, vp, vp], ci),
        "strassen_mlp_work_size": ([ci, ctypes.POINTER(ctypes.c_size_t)], ci),
        "strassen_mlp_loss_grad": ([vp, vp, vp, ci, vp, vp, vp, vp], ci),
        "strassen_mlp_adam": ([vp, vp, vp, vp, ci, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, vp], ci),
        "strassen_timing_enable": ([ci], ci),
        "strassen_timing_collect": ([ci, ctypes.POINTER(dbl), ctypes.POINTER(ci)], ci),
        "strassen_probe_rates": ([ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp], ci),
    }
    for name, (args, res) in specs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res


def last_error():
    return lib().strassen_last_error().decode()


def version():
    return lib().strassen_version().decode()


def check(rc):
    if rc != 0:
        raise StrassenError(rc, last_error())
    return rc


def header_functions():
    """Names of the functions include/strassen.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(strassen_[a-z0-9_]+)\s*\(", text)))


# ---------------------------------------------------------------------------------------------
# torch helpers
# ---------------------------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def colmajor(rows, cols, ld=None, device="cuda", dtype=None, fill=None):
    """Empty (or filled) column-major rows x cols tensor with leading dimension ld."""
    torch = _torch()
    dtype = dtype or torch.float64
    ld = rows if ld is None else ld
    buf = torch.empty((cols, max(ld, 1)), dtype=dtype, device=device)
    if fill is not None:
        buf.fill_(fill)
    return buf.t()[:rows, :]


def to_device(X, ld=None, device="cuda", offset=0):
    """Copy a 2-D numpy array into a column-major device tensor.  `offset` shifts the first
    element by that many doubles inside the allocation (to test unaligned operands)."""
    import numpy as np
    torch = _torch()
    X = np.asarray(X, dtype=np.float64)
    rows, cols = X.shape
    ld = rows if ld is None else ld
    flat = torch.zeros(offset + max(ld, 1) * cols, dtype=torch.float64, device=device)
    buf = flat[offset:].view(cols, max(ld, 1))
    buf[:, :rows] = torch.from_numpy(np.ascontiguousarray(X.T)).to(device)
    return buf.t()[:rows, :]


def to_host(T):
    """Column-major device tensor -> Fortran-order numpy array."""
    return T.t().contiguous().cpu().numpy().T


def _mat(T, name):
    torch = _torch()
    if T.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {T.dtype}")
    if T.dim() != 2:
        raise ValueError(f"{name}: expected a matrix")
    rows, cols = T.shape
    if rows > 1 and T.stride(0) != 1:
        raise ValueError(f"{name}: rows must be contiguous (column-major); got strides {T.stride()}")
    ld = T.stride(1)
    if cols <= 1:
        ld = max(ld, rows, 1)
    return T.data_ptr() if T.numel() > 0 else None, rows, cols, ld


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _variant(v):
    return VARIANTS[v] if isinstance(v, str) else int(v)


def dgemm(A, B, C, alpha=1.0, beta=1.0, levels=1, variant="abc", stream=None):
    """C := alpha*A*B + beta*C in place with `levels` levels of Strassen (0 = classical).
    A (m x k), B (k x n), C (m x n): float64 column-major device tensors."""
    pa, m, k, lda = _mat(A, "A")
    pb, k2, n, ldb = _mat(B, "B")
    pc, m2, n2, ldc = _mat(C, "C")
    if k2 != k or m2 != m or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    check(lib().strassen_dgemm(m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc, int(levels),
                               _variant(variant), _stream(stream)))
    return C


def gemm(A, B, C, alpha=1.0, beta=1.0, transa="N", transb="N", levels=-1, variant="abc",
         stream=None):
    """C := alpha*op(A)*op(B) + beta*C through strassen_gemm: op(X) = X ('N') or X^T ('T');
    A and B are the stored (untransposed) column-major matrices; levels = -1 lets the library
    choose the member."""
    pa, ra, ca, lda = _mat(A, "A")
    pb, rb, cb, ldb = _mat(B, "B")
    pc, m, n, ldc = _mat(C, "C")
    ta, tb = transa.upper() != "N", transb.upper() != "N"
    k = ra if ta else ca
    if (ca if ta else ra) != m or (cb if tb else rb) != k or (rb if tb else cb) != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)} ({transa}), B {tuple(B.shape)} "
                         f"({transb}), C {tuple(C.shape)}")
    check(lib().strassen_gemm(transa.encode(), transb.encode(), m, n, k, alpha, pa, lda, pb, ldb,
                              beta, pc, ldc, int(levels), _variant(variant), _stream(stream)))
    return C


def dgemm_winograd(A, B, C, alpha=1.0, beta=1.0, levels=1, stream=None):
    """C := alpha*A*B + beta*C with `levels` (1, 2) levels of Winograd's variant (ABC)."""
    pa, m, k, lda = _mat(A, "A")
    pb, k2, n, ldb = _mat(B, "B")
    pc, m2, n2, ldc = _mat(C, "C")
    if k2 != k or m2 != m or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    check(lib().strassen_dgemm_winograd(m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc,
                                        int(levels), _stream(stream)))
    return C


def workspace_size_winograd(m, n, k, levels):
    out = ctypes.c_size_t(0)
    check(lib().strassen_workspace_size_winograd(m, n, k, levels, ctypes.byref(out)))
    return out.value


def potrf_lower(A, nb=1024, levels=1, stream=None):
    """Cholesky factorization A = L L^T in place (strassen_dpotrf_lower): L overwrites the lower
    triangle of the square column-major device matrix A (the strict upper triangle is left as
    it is).  Returns info: 0, or j + 1 if the leading minor of order j + 1 is not positive
    definite."""
    a, m, n, lda = _mat(A, "A")
    if m != n:
        raise ValueError("A must be square")
    info = ctypes.c_int64(0)
    check(lib().strassen_dpotrf_lower(n, a, lda, int(nb), int(levels), ctypes.byref(info),
                                      _stream(stream)))
    return info.value


def getrf_nopiv(A, nb=1024, levels=1, stream=None):
    """LU factorization without pivoting of the square column-major device matrix A in place
    (unit lower L below the diagonal, U on and above), rank-nb updates with `levels` levels of
    Strassen (-1: the library chooses per update)."""
    pa, n, n2, lda = _mat(A, "A")
    if n2 != n:
        raise ValueError("square matrix expected")
    check(lib().strassen_dgetrf_nopiv(n, pa, lda, int(nb), int(levels), _stream(stream)))
    return A


def dgemm_noalloc(A, B, C, alpha=1.0, beta=1.0, levels=1, variant="abc", stream=None):
    """As :func:`dgemm`, through strassen_dgemm_noalloc: no device memory is allocated (the
    library's static scratch is the workspace)."""
    pa, m, k, lda = _mat(A, "A")
    pb, k2, n, ldb = _mat(B, "B")
    pc, m2, n2, ldc = _mat(C, "C")
    if k2 != k or m2 != m or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    check(lib().strassen_dgemm_noalloc(m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc,
                                       int(levels), _variant(variant), _stream(stream)))
    return C


NOALLOC_SCRATCH_BYTES = 256 << 20


def gemm_ex(A, B, C, alpha=1.0, beta=1.0, levels=1, compute="bf16", sum_prec="f64",
            c_prec="f64", variant="abc", stream=None):
    """Reduced-precision mode: products on BF16 MFMA (compute 'bf16' or 'bf16x3') with FP32
    accumulation, operand sums in `sum_prec`, C update in `c_prec`; A, B, C are FP64."""
    pa, m, k, lda = _mat(A, "A")
    pb, k2, n, ldb = _mat(B, "B")
    pc, m2, n2, ldc = _mat(C, "C")
    if k2 != k or m2 != m or n2 != n:
        raise ValueError("shape mismatch")
    check(lib().strassen_gemm_ex(m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc, int(levels),
                                 _variant(variant), COMPUTE[compute], PREC[sum_prec], PREC[c_prec],
                                 _stream(stream)))
    return C


def raw_dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant, stream=None):
    """Direct call with integer pointers; returns the library's status code (no raise)."""
    return lib().strassen_dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant,
                                stream)


def workspace_size(m, n, k, levels, variant):
    out = ctypes.c_size_t(0)
    check(lib().strassen_workspace_size(m, n, k, levels, _variant(variant), ctypes.byref(out)))
    return out.value


def workspace_size_ex(m, n, k, levels, compute):
    out = ctypes.c_size_t(0)
    check(lib().strassen_workspace_size_ex(m, n, k, levels, COMPUTE[compute], ctypes.byref(out)))
    return out.value


def set_workspace(tensor_or_none):
    """Use a caller-owned device buffer (a torch tensor, kept alive by the caller) as workspace;
    None returns to the library's own."""
    if tensor_or_none is None:
        check(lib().strassen_set_workspace(None, 0))
    else:
        t = tensor_or_none
        check(lib().strassen_set_workspace(t.data_ptr(), t.numel() * t.element_size()))


def set_workspace_limit(nbytes):
    """Cap the library-owned workspace at `nbytes` (0 or None: no cap)."""
    check(lib().strassen_set_workspace_limit(int(nbytes or 0)))


def set_tile_config(cfg):
    """Force a kernel / tile configuration (0..5, see strassen.h) for later calls, or -1 for the
    automatic choice."""
    check(lib().strassen_set_tile_config(int(cfg)))


KERNEL_KINDS = {"all_products": 0, "outer_sums": 1, "tile": 2, "bf16": 3, "cast": 4, "pad": 5,
                "classical": 6}


def probe_rates(stream=None):
    """Measured FP64 and BF16 matrix-core issue rates (TFLOP/s) of the current device."""
    f, b = ctypes.c_double(), ctypes.c_double()
    check(lib().strassen_probe_rates(ctypes.byref(f), ctypes.byref(b), _stream(stream)))
    return f.value, b.value


def timing_enable(on=True):
    """Record HIP events around every later launch of the library's main kernels."""
    check(lib().strassen_timing_enable(1 if on else 0))


def timing_collect(kind):
    """(total milliseconds, launches) of the recorded launches of one kernel kind (a key of
    KERNEL_KINDS), which are then forgotten; waits for them."""
    ms, cnt = ctypes.c_double(), ctypes.c_int()
    check(lib().strassen_timing_collect(KERNEL_KINDS[kind], ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def release_workspace():
    check(lib().strassen_release_workspace())


def table(levels):
    """The operation table the kernels execute: list of (A terms, B terms, C terms), each term
    ((row_block, col_block), sign)."""
    L = lib()
    nprod = L.strassen_table_size(levels)
    if nprod < 0:
        raise ValueError("levels out of range")
    q = 2 ** levels
    out = []
    for r in range(nprod):
        na, nb, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        a, b, c = (ctypes.c_int * 8)(), (ctypes.c_int * 8)(), (ctypes.c_int * 8)()
        check(L.strassen_table_get(levels, r, ctypes.byref(na), a, ctypes.byref(nb), b,
                                   ctypes.byref(nc), c))

        def dec(v):
            s = 1 if v > 0 else -1
            v = abs(v) - 1
            return ((v % q, v // q), s)
        out.append(([dec(a[i]) for i in range(na.value)], [dec(b[i]) for i in range(nb.value)],
                    [dec(c[i]) for i in range(nc.value)]))
    return out


# ---------------------------------------------------------------------------------------------
# batched mode
# ---------------------------------------------------------------------------------------------
class Batched:
    """A batch of independent FP64 GEMMs run by one persistent kernel (see strassen.h).

    shapes: list of (m, n, k); levels / cfg: per-problem lists with -1 = library choice
    (None = all -1); cfg 0 / 1: 128 x 128 / 64 x 64 tiles of the persistent kernel, 2: the
    problem's own all-products launch(es), 3: its own single-call launches on a side stream."""

    def __init__(self, shapes, levels=None, cfg=None):
        self.count = len(shapes)
        i64 = ctypes.c_int64 * max(1, self.count)
        ci = ctypes.c_int * max(1, self.count)
        self._m = i64(*[s[0] for s in shapes])
        self._n = i64(*[s[1] for s in shapes])
        self._k = i64(*[s[2] for s in shapes])
        lv = ci(*(levels if levels is not None else [-1] * self.count))
        cf = ci(*(cfg if cfg is not None else [-1] * self.count))
        self._plan = ctypes.c_void_p()
        check(lib().strassen_batched_plan(self.count, self._m, self._n, self._k, lv, cf,
                                          ctypes.byref(self._plan)))

    def autotune(self, sample=64, seed=0, stream=None):
        check(lib().strassen_batched_autotune(self._plan, int(sample), int(seed), _stream(stream)))

    def choices(self):
        out = []
        for i in range(self.count):
            lv, cf = ctypes.c_int(), ctypes.c_int()
            check(lib().strassen_batched_choice(self._plan, i, ctypes.byref(lv), ctypes.byref(cf)))
            out.append((lv.value, cf.value))
        return out

    def _operands(self, As, Bs, Cs):
        vp = ctypes.c_void_p * max(1, self.count)
        i64 = ctypes.c_int64 * max(1, self.count)
        pa, pb, pc, la, lb, lc = [], [], [], [], [], []
        for A, B, C in zip(As, Bs, Cs):
            a, _, _, lda = _mat(A, "A")
            b, _, _, ldb = _mat(B, "B")
            c, _, _, ldc = _mat(C, "C")
            pa.append(a); pb.append(b); pc.append(c)
            la.append(lda); lb.append(ldb); lc.append(ldc)
        self._keep = (vp(*pa), i64(*la), vp(*pb), i64(*lb), vp(*pc), i64(*lc))
        return self._keep

    def run(self, As, Bs, Cs, alpha=1.0, beta=1.0, stream=None):
        a, la, b, lb, c, lc = self._operands(As, Bs, Cs)
        check(lib().strassen_batched_run(self._plan, a, la, b, lb, c, lc, alpha, beta,
                                         _stream(stream)))

    def capture(self, As, Bs, Cs, alpha=1.0, beta=1.0, stream=None):
        a, la, b, lb, c, lc = self._operands(As, Bs, Cs)
        check(lib().strassen_batched_capture(self._plan, a, la, b, lb, c, lc, alpha, beta,
                                             _stream(stream)))

    def replay(self, stream=None):
        check(lib().strassen_batched_replay(self._plan, _stream(stream)))

    def close(self):
        if self._plan:
            check(lib().strassen_batched_destroy(self._plan))
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

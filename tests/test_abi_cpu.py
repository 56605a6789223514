"""Host-side checks of the C-ABI library (no GPU needed, no compute calls).

The library must load, export every function include/strassen.h declares, reject invalid
arguments with the documented -i codes before touching any device, report workspace sizes
that follow from the sub-block shapes, and carry the same operation tables as the oracle.
"""
import ctypes

import numpy as np
import pytest

import paper_1605_01078_amd as sx
from oracle import tables as otab


def test_library_loads_and_exports_header_functions():
    L = sx.lib()
    names = sx.header_functions()
    assert "strassen_dgemm" in names and "strassen_gemm_ex" in names
    for name in names:
        assert hasattr(L, name), name
    assert "gfx950" in sx.version()


BAD = [
    # (m, n, k, lda, ldb, ldc, levels, variant, A, B, C) -> expected code
    ((-1, 4, 4, 4, 4, 4, 1, 0, 1, 1, 1), -1),
    ((4, -1, 4, 4, 4, 4, 1, 0, 1, 1, 1), -2),
    ((4, 4, -1, 4, 4, 4, 1, 0, 1, 1, 1), -3),
    ((4, 4, 4, 4, 4, 4, 1, 0, 0, 1, 1), -5),
    ((4, 4, 4, 3, 4, 4, 1, 0, 1, 1, 1), -6),
    ((4, 4, 4, 4, 4, 4, 1, 0, 1, 0, 1), -7),
    ((4, 4, 5, 4, 4, 4, 1, 0, 1, 1, 1), -8),
    ((4, 4, 4, 4, 4, 4, 1, 0, 1, 1, 0), -10),
    ((4, 4, 4, 4, 4, 3, 1, 0, 1, 1, 1), -11),
    ((4, 4, 4, 4, 4, 4, 4, 0, 1, 1, 1), -12),
    ((4, 4, 4, 4, 4, 4, 3, 1, 1, 1, 1), -13),    # three levels: ABC only
    ((4, 4, 4, 4, 4, 4, 3, 2, 1, 1, 1), -13),
    ((4, 4, 4, 4, 4, 4, -1, 0, 1, 1, 1), -12),
    ((4, 4, 4, 4, 4, 4, 1, 3, 1, 1, 1), -13),
    ((0, 4, 4, 0, 4, 0, 1, 0, 1, 1, 1), -6),     # lda >= max(1, m) even when m == 0
]


@pytest.mark.parametrize("args,code", BAD)
def test_invalid_arguments(args, code):
    m, n, k, lda, ldb, ldc, lev, var, pa, pb, pc = args
    fake = 1 << 20   # never dereferenced: validation fails first
    rc = sx.raw_dgemm(m, n, k, 1.0, fake * pa or None, lda, fake * pb or None, ldb, 1.0,
                      fake * pc or None, ldc, lev, var, None)
    assert rc == code
    assert sx.last_error() != ""


def test_quick_return_without_device():
    # m == 0 or n == 0: nothing to do, success, no device touched (none exists here)
    assert sx.raw_dgemm(0, 5, 5, 1.0, None, 1, None, 5, 1.0, None, 1, 1, 0, None) == 0
    assert sx.raw_dgemm(5, 0, 5, 1.0, None, 5, None, 5, 1.0, None, 5, 2, 1, None) == 0


def test_null_operands_allowed_when_not_read():
    # alpha == 0: A and B are not referenced (BLAS); with m == 0 nothing at all is done
    assert sx.raw_dgemm(0, 3, 3, 0.0, None, 1, None, 3, 1.0, None, 1, 1, 0, None) == 0


@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_tables_match_oracle(levels):
    lib_tab = sx.table(levels)
    ora = otab.table(levels)
    assert len(lib_tab) == len(ora)
    for r, (la, lb, lc) in enumerate(lib_tab):
        oa, ob, oc = ora[r]
        assert la == [tuple(t) for t in oa], r
        assert lb == [tuple(t) for t in ob], r
        assert sorted(lc) == sorted(tuple(t) for t in oc), r


def test_tables_satisfy_identity():
    for levels in (1, 2, 3):
        tab = sx.table(levels)
        assert np.array_equal(otab.tensor_of(tab, levels), otab.matmul_tensor(levels))


def _cdiv(a, b):
    return -(-a // b)


def _one_level_staged(m, n, k):
    """The shapes on which one-level ABC stages its sums and runs the classical kernel: exact
    quadrants, k/2 >= 2048, whole rounds of 256 x 128 tiles (95% of the last one) and either
    k/2 >= 4096 or at least 1024 tiles."""
    if m % 4 or k % 4 or n % 2:
        return False
    tiles = _cdiv(m // 2, 256) * _cdiv(n // 2, 128)
    rounds = _cdiv(tiles, 256)
    return tiles >= 256 and k // 2 >= 2048 and 20 * tiles >= 19 * 256 * rounds and \
        (k // 2 >= 4096 or tiles >= 1024)


def test_one_level_staged_shapes():
    assert _one_level_staged(16384, 16384, 16384) and _one_level_staged(8192, 8192, 8192)
    assert not _one_level_staged(16384, 16384, 2048)    # rank-k: the all-products kernel
    assert not _one_level_staged(12288, 12288, 12288)   # 4.5 rounds of tiles
    r32 = lambda x: _cdiv(x, 32) * 32
    for m, n, k in [(16384, 16384, 4096), (8192, 8192, 8192), (8188, 8190, 8196),
                    (16384, 16384, 2048), (12288, 12288, 12288), (8192, 8192, 4096)]:
        want = 8 * (5 * r32((m // 2) * (k // 2)) + 5 * r32((k // 2) * (n // 2)))
        assert sx.workspace_size(m, n, k, 1, "abc") == (want if _one_level_staged(m, n, k) else 0)


@pytest.mark.parametrize("m,n,k", [(512, 512, 512), (1000, 777, 333), (16384, 16384, 16384)])
def test_workspace_sizes(m, n, k):
    assert sx.workspace_size(m, n, k, 0, "ab") == 0
    for levels in (1, 2):
        q = 2 ** levels
        mq, nq, kq = _cdiv(m, q), _cdiv(n, q), _cdiv(k, q)
        if levels == 1 or m < 4096:   # two-level staging: test_two_level_abc_staging_workspace
            # block-padded copies where m or k is not a multiple of 2^(L+1): A as mp x kp and B
            # as kp x n (C too if m needs it), every sub-block extent rounded up to even
            u = 2 * q
            mp, kp = q * 2 * _cdiv(mq, 2), q * 2 * _cdiv(kq, 2)
            r32 = lambda x: _cdiv(x, 32) * 32
            want = 0
            if m % u or k % u:
                want = 8 * (r32(mp * kp) + r32(kp * n) + (r32(mp * n) if m % u else 0))
            elif levels == 1 and _one_level_staged(m, n, k):
                # one level staged on the classical kernel: five A and five B quadrant sums
                want = 8 * (5 * r32(mq * kq) + 5 * r32(kq * nq))
            assert sx.workspace_size(m, n, k, levels, "abc") == want
        ab = sx.workspace_size(m, n, k, levels, "ab")
        nprod = 7 ** levels
        # one M_r per product, leading dimension rounded to 8 doubles, slot to 32; AB on the
        # all-products kernel adds block-padded A and B copies where m or k is not a multiple of
        # 2^(L+1) and, at two levels, the staged outer sums (where two-level ABC would stage)
        per = _cdiv(_cdiv(mq, 8) * 8 * nq, 32) * 32
        r32 = lambda x: _cdiv(x, 32) * 32
        u = 2 * q
        mp, kp = q * 2 * _cdiv(mq, 2), q * 2 * _cdiv(kq, 2)
        staged = levels == 2 and (mp // 2) * (_cdiv(n, 4) * 2) >= 2048 ** 2 and kp >= 2048
        # copies are made only where a launch has at least 192 tile positions of 64 x 64
        positions = _cdiv(2 * _cdiv(mq, 2), 64) * _cdiv(nq, 64)
        copies = bool(m % u or k % u or (staged and n % 4))
        extra = 0
        if (levels == 1 or staged) and (not copies or positions >= 192):
            np_ = 4 * nq if staged and n % 4 else n
            if m % u or k % u:
                extra += 8 * r32(mp * kp)
            if k % u or np_ != n:
                extra += 8 * r32(kp * np_)
            if staged:
                extra += 8 * (5 * r32((mp // 2) * (kp // 2)) + 5 * r32((kp // 2) * (np_ // 2)))
        assert ab == 8 * nprod * per + extra
        ab -= extra
        nv = sx.workspace_size(m, n, k, levels, "naive")
        tab = otab.table(levels)
        na = sum(1 for a, _, _ in tab if len(a) > 1 or a[0][1] < 0)
        nb = sum(1 for _, b, _ in tab if len(b) > 1 or b[0][1] < 0)
        assert (na, nb) == ((5, 5) if levels == 1 else (45, 45))
        assert nv == ab + 8 * (na * _cdiv(mq * kq, 32) * 32 + nb * _cdiv(kq * nq, 32) * 32)


def test_two_level_abc_staging_workspace():
    """Two-level ABC reports the staging buffers of its outer operand sums (five A sums of
    m/2 x k/2 and five B sums of k/2 x n/2, slots rounded to 32 doubles) where staging applies:
    n a multiple of 4, outer C blocks of at least 2048 x 2048 and k >= 2048."""
    r32 = lambda x: _cdiv(x, 32) * 32
    for m, n, k in [(16384, 16384, 16384), (4096, 4096, 4096), (8192, 12288, 2048)]:
        want = 8 * (5 * r32((m // 2) * (k // 2)) + 5 * r32((k // 2) * (n // 2)))
        assert sx.workspace_size(m, n, k, 2, "abc") == want
        # one level: its own staged sums where its products fill the GPU on the classical kernel
        h = 8 * (5 * r32((m // 2) * (k // 2)) + 5 * r32((k // 2) * (n // 2)))
        assert sx.workspace_size(m, n, k, 1, "abc") == (h if _one_level_staged(m, n, k) else 0)
    for m, n, k in [(2048, 4096, 4096), (8192, 8192, 1024)]:
        assert sx.workspace_size(m, n, k, 2, "abc") == 0
    # n not a multiple of 4: B and C are copied with n rounded up to 4 columns, then staged
    m, n, k = 8192, 8190, 8192
    n4 = 4 * _cdiv(n, 4)
    want = 8 * (r32(k * n4) + r32(m * n4) + 5 * r32((m // 2) * (k // 2)) + 5 * r32((k // 2) * (n4 // 2)))
    assert sx.workspace_size(m, n, k, 2, "abc") == want


def test_workspace_size_errors():
    out = ctypes.c_size_t()
    L = sx.lib()
    assert L.strassen_workspace_size(-1, 1, 1, 1, 0, ctypes.byref(out)) == -1
    assert L.strassen_workspace_size(1, 1, 1, 5, 0, ctypes.byref(out)) == -4
    assert L.strassen_workspace_size(1, 1, 1, 1, 9, ctypes.byref(out)) == -5
    assert L.strassen_set_workspace(ctypes.c_void_p(8), 64) == -1
    assert L.strassen_set_workspace(ctypes.c_void_p(256), 0) == -2
    assert L.strassen_set_workspace(None, 0) == 0


def test_gemm_ex_argument_checks():
    L = sx.lib()
    p = ctypes.c_void_p(256)   # never dereferenced: every call below fails its checks first
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, p, 4, p, 4, 1.0, p, 4, 1, 0, 7, 0, 0, None)
    assert rc == -14
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, p, 4, p, 4, 1.0, p, 4, 1, 0, 1, 2, 0, None)
    assert rc == -15
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, p, 4, p, 4, 1.0, p, 4, 1, 0, 1, 0, 5, None)
    assert rc == -16
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, p, 4, p, 4, 1.0, p, 4, 1, 1, 1, 0, 0, None)
    assert rc == -13          # the reduced-precision mode is ABC only
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, None, 4, p, 4, 1.0, p, 4, 1, 0, 1, 0, 0, None)
    assert rc == -5
    rc = L.strassen_gemm_ex(4, 4, 4, 1.0, p, 4, p, 4, 1.0, p, 4, 3, 0, 1, 0, 0, None)
    assert rc == -12
    # m == 0: quick return before any device work
    assert L.strassen_gemm_ex(0, 4, 4, 1.0, p, 1, p, 4, 1.0, p, 1, 1, 0, 1, 0, 0, None) == 0


@pytest.mark.parametrize("m,n,k", [(512, 512, 512), (1000, 777, 333), (8192, 8192, 8192)])
def test_workspace_size_ex(m, n, k):
    for levels in (0, 1, 2):
        q = 2 ** levels
        mp = _cdiv(_cdiv(m, q), 128) * 128
        np_ = _cdiv(_cdiv(n, q), 128) * 128
        kp = _cdiv(_cdiv(k, q), 64) * 64
        nprod = 7 ** levels
        assert sx.workspace_size_ex(m, n, k, levels, "f64") == 0
        assert sx.workspace_size_ex(m, n, k, levels, "bf16") == 2 * nprod * (mp + np_) * kp
        assert sx.workspace_size_ex(m, n, k, levels, "bf16x3") == 4 * nprod * (mp + np_) * kp
    out = ctypes.c_size_t()
    assert sx.lib().strassen_workspace_size_ex(1, 1, 1, 1, 3, ctypes.byref(out)) == -5


def test_ab_padded_workspace():
    """AB on the all-products kernel reports its block-padded A and B copies (A as mp x kp, B as
    kp x n', every sub-block extent rounded up to even, n' = n rounded up to 4 where two-level
    staging needs it) and the staged outer sums of the padded problem behind the product
    temporaries, where a launch has at least 192 tile positions; two levels without staging and
    smaller padded problems run the tile kernel and need the temporaries only."""
    r32 = lambda x: _cdiv(x, 32) * 32

    def temps(m, n, levels):
        q = 2 ** levels
        return 8 * 7 ** levels * r32(_cdiv(_cdiv(m, q), 8) * 8 * _cdiv(n, q))

    # one level, m and k not multiples of 4: both operands copied (528 tile positions)
    m, n, k = 3001, 2777, 1333
    mp, kp = 2 * 2 * _cdiv(_cdiv(m, 2), 2), 2 * 2 * _cdiv(_cdiv(k, 2), 2)
    assert sx.workspace_size(m, n, k, 1, "ab") == temps(m, n, 1) + 8 * (r32(mp * kp) + r32(kp * n))
    # one level, only k ragged in the sense of the layout (k % 4 == 2): A and B copied
    m, n, k = 3000, 2777, 1026
    kp = 2 * 2 * _cdiv(_cdiv(k, 2), 2)
    assert sx.workspace_size(m, n, k, 1, "ab") == temps(m, n, 1) + 8 * (r32(m * kp) + r32(kp * n))
    # fewer than 192 tile positions of 64 x 64 per launch (here 56): no copies, the tile kernel
    assert sx.workspace_size(1001, 777, 333, 1, "ab") == temps(1001, 777, 1)
    # but operands that fit the layout run the fused kernel at any size, with no copies
    assert sx.workspace_size(1000, 776, 332, 1, "ab") == temps(1000, 776, 1)
    # two levels staged, n % 4 == 2: B copied with n rounded up to 4, A used in place
    m, n, k = 8192, 8190, 8192
    n4 = 4 * _cdiv(n, 4)
    want = temps(m, n, 2) + 8 * (r32(k * n4) + 5 * r32((m // 2) * (k // 2)) + 5 * r32((k // 2) * (n4 // 2)))
    assert sx.workspace_size(m, n, k, 2, "ab") == want
    # two levels where staging does not apply: the tile kernel, temporaries only
    for m, n, k in [(1001, 777, 333), (2048, 4096, 4096)]:
        assert sx.workspace_size(m, n, k, 2, "ab") == temps(m, n, 2)


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


TILE_LD = 2 ** 21 - 1   # 8 * 128 * (ld + 1) reaches 2^31: the tile kernel's lane offsets overflow


@pytest.mark.parametrize("levels,variant,which", [
    (0, 0, "ldb"), (0, 0, "ldc"), (0, 0, "lda"),        # classical: the tile kernel
    (1, 2, "lda"), (2, 2, "ldb"),                        # Naive: tile kernel over temporaries
    (1, 1, "ldb"),                                        # AB below 192 positions: tile kernel
])
def test_tile_kernel_offset_guard_is_host_side(levels, variant, which):
    """Leading dimensions whose 128 columns span 2 GiB are refused with STRASSEN_ERR_UNSUPPORTED
    on every path that runs the general tile kernel, before any device call (this machine may
    have no GPU: the code must not be STRASSEN_ERR_NO_DEVICE)."""
    m = n = k = 64
    ld = {"lda": m, "ldb": k, "ldc": m}
    ld[which] = TILE_LD
    fake = 1 << 20   # never dereferenced: the call is refused on the host
    rc = sx.raw_dgemm(m, n, k, 1.0, fake, ld["lda"], fake, ld["ldb"], 1.0, fake, ld["ldc"],
                      levels, variant, None)
    assert rc == 3, (rc, sx.last_error())
    assert "tile kernel" in sx.last_error()


@pytest.mark.skipif(not _no_gpu(), reason="with a GPU this call would launch on fake pointers")
def test_tile_kernel_offset_guard_boundary():
    """One below the limit the call passes the host checks and reaches the device check."""
    fake = 1 << 20
    rc = sx.raw_dgemm(64, 64, 64, 1.0, fake, 64, fake, TILE_LD - 1, 1.0, fake, 64, 0, 0, None)
    assert rc == 4, (rc, sx.last_error())   # STRASSEN_ERR_NO_DEVICE on a machine without GPU


def test_workspace_limit_entry_point():
    L = sx.lib()
    assert L.strassen_set_workspace_limit(1 << 20) == 0
    assert L.strassen_set_workspace_limit(0) == 0   # no cap


def test_three_level_workspace():
    """Three levels stage the sums of the two upper levels: five slots per side of m/2 x k/2 and
    k/2 x n/2, and five of m/4 x k/4 and k/4 x n/4 reused from one top-level product to the next
    (each rounded up to 32 doubles); ragged sizes add block-padded copies (every level-3 sub-block
    extent even, n rounded up to 8)."""
    r32 = lambda x: _cdiv(x, 32) * 32
    m = n = k = 4096
    want = 8 * 5 * (r32(2048 * 2048) * 2 + r32(1024 * 1024) * 2)
    assert sx.workspace_size(m, n, k, 3, "abc") == want
    m, n, k = 1000, 999, 1001
    mp, kp, np_ = 8 * 2 * _cdiv(_cdiv(m, 8), 2), 8 * 2 * _cdiv(_cdiv(k, 8), 2), 8 * _cdiv(n, 8)
    want = 8 * (r32(mp * kp) + r32(kp * np_) + r32(mp * np_) +
                5 * (r32(mp // 2 * kp // 2) + r32(kp // 2 * np_ // 2)) +
                5 * (r32(mp // 4 * kp // 4) + r32(kp // 4 * np_ // 4)))
    assert sx.workspace_size(m, n, k, 3, "abc") == want
    out = ctypes.c_size_t()
    assert sx.lib().strassen_workspace_size(64, 64, 64, 3, 1, ctypes.byref(out)) == -5


def test_winograd_entry_point_checks_and_workspace():
    L = sx.lib()
    fake = 1 << 20
    for levels in (0, 3):
        assert L.strassen_dgemm_winograd(64, 64, 64, 1.0, fake, 64, fake, 64, 1.0, fake, 64,
                                         levels, None) == -12
    assert L.strassen_dgemm_winograd(64, 64, 64, 1.0, fake, 63, fake, 64, 1.0, fake, 64, 1,
                                     None) == -6
    r32 = lambda x: _cdiv(x, 32) * 32
    assert sx.workspace_size_winograd(4096, 4096, 4096, 1) == 0
    # one level where its products run on the classical kernel: the eight staged chain sums
    assert sx.workspace_size_winograd(16384, 16384, 16384, 1) == 8 * 8 * r32(8192 * 8192)
    assert sx.workspace_size_winograd(16384, 16384, 2048, 1) == 0
    assert sx.workspace_size_winograd(4096, 4096, 4096, 2) == 8 * 8 * r32(2048 * 2048)
    m, n, k = 1001, 998, 777
    mp, kp = 2 * 2 * _cdiv(_cdiv(m, 2), 2), 2 * 2 * _cdiv(_cdiv(k, 2), 2)
    assert sx.workspace_size_winograd(m, n, k, 1) == 8 * (r32(mp * kp) + r32(kp * n) + r32(mp * n))


def test_getrf_argument_codes():
    L = sx.lib()
    fake = 1 << 20
    assert L.strassen_dgetrf_nopiv(-1, fake, 4, 64, 0, None) == -1
    assert L.strassen_dgetrf_nopiv(4, None, 4, 64, 0, None) == -2
    assert L.strassen_dgetrf_nopiv(4, fake, 3, 64, 0, None) == -3
    assert L.strassen_dgetrf_nopiv(4, fake, 4, 100, 0, None) == -4
    assert L.strassen_dgetrf_nopiv(4, fake, 4, 0, 0, None) == -4
    assert L.strassen_dgetrf_nopiv(4, fake, 4, 64, 4, None) == -5
    assert L.strassen_dgetrf_nopiv(0, None, 1, 64, 0, None) == 0


def test_potrf_argument_errors():
    """strassen_dpotrf_lower rejects bad arguments on the host (no device needed)."""
    L = sx.lib()
    info = ctypes.c_int64(-7)
    buf = (ctypes.c_double * 64)()
    assert L.strassen_dpotrf_lower(-1, buf, 8, 64, 0, ctypes.byref(info), None) == -1
    assert L.strassen_dpotrf_lower(8, None, 8, 64, 0, ctypes.byref(info), None) == -2
    assert L.strassen_dpotrf_lower(8, buf, 7, 64, 0, ctypes.byref(info), None) == -3
    assert L.strassen_dpotrf_lower(8, buf, 8, 48, 0, ctypes.byref(info), None) == -4
    assert L.strassen_dpotrf_lower(8, buf, 8, 0, 0, ctypes.byref(info), None) == -4
    assert L.strassen_dpotrf_lower(8, buf, 8, 64, 4, ctypes.byref(info), None) == -5
    assert L.strassen_dpotrf_lower(0, None, 1, 64, 0, ctypes.byref(info), None) == 0
    assert info.value == 0
    assert L.strassen_dpotrf_lower(0, None, 1, 64, 0, None, None) == 0

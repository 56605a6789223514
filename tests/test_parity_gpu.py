"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every call goes through the C-ABI (via the ctypes binding).  Tolerances:
  * small integer inputs: bit-exact (every intermediate of one- and two-level Strassen is an
    integer below 2^53, so any order of exact operations gives the same value);
  * real inputs, Strassen: relative Frobenius error <= 1e-12 (one level), 1e-11 (two levels)
    against the plain-definition oracle;
  * real inputs, classical: elementwise |C - C_ref| <= 2 gamma_{k+2} (|alpha||A||B| + |beta||C|),
    the rounding-error bound of any summation order (Higham, Sec. 3.1).
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, oracle_strassen, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
TOL = {1: 1e-12, 2: 1e-11}
VARIANTS = ["abc", "ab", "naive"]


def run(A, B, C, alpha, beta, levels, variant, lda=None, ldb=None, ldc=None, offset=0):
    dA = sx.to_device(A, ld=lda, offset=offset)
    dB = sx.to_device(B, ld=ldb, offset=offset)
    dC = sx.to_device(C, ld=ldc, offset=offset)
    sx.dgemm(dA, dB, dC, alpha, beta, levels, variant)
    torch.cuda.synchronize()
    return sx.to_host(dC)


def classical_bound(A, B, C, alpha, beta):
    k = A.shape[1]
    g = (k + 2) * U / (1 - (k + 2) * U)
    return 2 * g * (abs(alpha) * (np.abs(A) @ np.abs(B)) + abs(beta) * np.abs(C))


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("variant", VARIANTS)
def test_c1_uniform_512(levels, variant):
    if levels == 0 and variant != "abc":
        pytest.skip("classical has one variant")
    print(f"case c1 uniform L={levels} {variant}", flush=True)
    A, B, C = W.problem(0, 512, 512, 512, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    got = run(A, B, C, 1.0, 1.0, levels, variant)
    if levels == 0:
        assert np.all(np.abs(got - ref) <= classical_bound(A, B, C, 1.0, 1.0))
    else:
        assert rel_fro(got, ref) <= TOL[levels]


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("variant", VARIANTS)
def test_c1_integer_bit_exact(levels, variant):
    print(f"case c1 integer L={levels} {variant}", flush=True)
    A, B, C = W.problem(0, 512, 512, 512, "integer", c_zero=True)
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    if levels > 0:
        ref2 = oracle_strassen(A, B, C.copy(order="F"), 1.0, 1.0, levels)
        assert np.array_equal(ref, ref2)
    got = run(A, B, C, 1.0, 1.0, levels, variant)
    assert np.array_equal(got, ref)


RAGGED = [(1, 1, 1), (3, 5, 7), (17, 33, 9), (255, 257, 130), (513, 511, 515), (1000, 1000, 1000),
          (64, 1030, 31), (700, 90, 1290), (129, 2, 260)]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_ragged_integer_all_variants(shape, levels):
    m, n, k = shape
    print(f"case ragged integer {shape} L={levels}", flush=True)
    A, B, C = W.problem(1, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 2.0, -1.0)
    outs = []
    for variant in (VARIANTS if levels else ["abc"]):
        got = run(A, B, C, 2.0, -1.0, levels, variant)
        assert np.array_equal(got, ref), variant
        outs.append(got)


@pytest.mark.parametrize("shape", [(255, 257, 130), (513, 511, 515), (1000, 777, 333)])
@pytest.mark.parametrize("levels", [1, 2])
def test_ragged_uniform_tolerance_and_variants_bitwise(shape, levels):
    m, n, k = shape
    print(f"case ragged uniform {shape} L={levels}", flush=True)
    A, B, C = W.problem(2, m, n, k, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 0.75, 0.5)
    outs = [run(A, B, C, 0.75, 0.5, levels, v) for v in VARIANTS]
    for got in outs:
        assert rel_fro(got, ref) <= TOL[levels]
    # same table, same product order, same update arithmetic: variants agree bit for bit
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_leading_dimensions_and_unaligned(levels):
    m, n, k = 300, 260, 270
    print(f"case ld/unaligned L={levels}", flush=True)
    A, B, C = W.problem(3, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    for lda, ldb, ldc, off in [(m + 3, k + 5, m + 1, 0), (m + 8, k + 8, m + 8, 1), (m, k, m, 1)]:
        got = run(A, B, C, 1.0, 1.0, levels, "abc", lda, ldb, ldc, off)
        assert np.array_equal(got, ref), (lda, ldb, ldc, off)


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("variant", VARIANTS)
def test_beta_zero_ignores_nan_in_c(levels, variant):
    A, B, _ = W.problem(4, 130, 140, 150, "integer")
    C = np.full((130, 140), np.nan, order="F")
    got = run(A, B, C, 1.0, 0.0, levels, variant)
    ref = oracle_dgemm(A, B, np.zeros((130, 140), order="F"), 1.0, 0.0)
    assert np.array_equal(got, ref)


def test_alpha_zero_and_k_zero_scale_c_only():
    g = np.random.default_rng(5)
    C = W.integers(g, 70, 90)
    A = np.full((70, 40), np.nan, order="F")
    B = np.full((40, 90), np.nan, order="F")
    for levels in (0, 1, 2):
        got = run(A, B, C, 0.0, 3.0, levels, "abc")
        assert np.array_equal(got, 3.0 * C)
        got = run(A, B, C, 0.0, 0.0, levels, "ab")
        assert np.all(got == 0.0)
    dA = sx.colmajor(70, 0)
    dB = sx.colmajor(0, 90)
    dC = sx.to_device(C)
    sx.dgemm(dA, dB, dC, 1.0, -2.0, 1, "abc")
    torch.cuda.synchronize()
    assert np.array_equal(sx.to_host(dC), -2.0 * C)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_determinism_and_power_of_two_scaling(levels):
    A, B, C = W.problem(6, 600, 520, 700, "uniform")
    a1 = run(A, B, C, 1.0, 0.0, levels, "abc")
    a2 = run(A, B, C, 1.0, 0.0, levels, "abc")
    assert np.array_equal(a1, a2)
    a3 = run(2.0 * A, B, C, 1.0, 0.0, levels, "abc")
    assert np.array_equal(a3, 2.0 * a1)
    a4 = run(A, B, C, 0.5, 0.0, levels, "abc")
    assert np.array_equal(a4, 0.5 * a1)


@pytest.mark.parametrize("levels", [1, 2])
def test_strassen_error_comparable_to_oracle_strassen(levels):
    A, B, C = W.problem(7, 512, 512, 512, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    o2 = oracle_strassen(A, B, C.copy(order="F"), 1.0, 1.0, levels)
    got = run(A, B, C, 1.0, 1.0, levels, "abc")
    e_gpu, e_o2 = rel_fro(got, ref), rel_fro(o2, ref)
    print(f"L={levels}: gpu {e_gpu:.3e} oracle-strassen {e_o2:.3e}")
    assert e_gpu <= 10 * e_o2 + 1e-16


def test_caller_workspace():
    A, B, C = W.problem(8, 400, 300, 200, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    need = sx.workspace_size(400, 300, 200, 2, "naive")
    ws = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
    sx.set_workspace(ws)
    try:
        assert np.array_equal(run(A, B, C, 1.0, 1.0, 2, "naive"), ref)
        small = torch.empty(64, dtype=torch.float64, device="cuda")
        sx.set_workspace(small)
        dA, dB, dC = sx.to_device(A), sx.to_device(B), sx.to_device(C)
        with pytest.raises(sx.StrassenError) as ei:
            sx.dgemm(dA, dB, dC, 1.0, 1.0, 2, "ab")
        assert ei.value.code == 2
        torch.cuda.synchronize()
        assert np.array_equal(sx.to_host(dC), C)   # untouched
    finally:
        sx.set_workspace(None)


@pytest.mark.parametrize("levels", [1, 2])
def test_workspace_limit_abc_falls_back_ab_refuses(levels):
    """A cap on the library-owned workspace below what the block-padded copies (ragged shape)
    need: ABC runs its workspace-free path and gives the same bits; AB, whose temporaries the
    cap does not allow, fails with STRASSEN_ERR_ALLOC and leaves C untouched."""
    m, n, k = 300, 260, 270
    print(f"case workspace limit L={levels}", flush=True)
    A, B, C = W.problem(12, m, n, k, "uniform")
    free = run(A, B, C, 0.5, -1.5, levels, "abc")
    sx.release_workspace()
    sx.set_workspace_limit(4096)
    try:
        capped = run(A, B, C, 0.5, -1.5, levels, "abc")
        assert np.array_equal(capped, free)
        Ai, Bi, Ci = W.problem(13, m, n, k, "integer")
        ref = oracle_dgemm(Ai, Bi, Ci.copy(order="F"), 1.0, 1.0)
        assert np.array_equal(run(Ai, Bi, Ci, 1.0, 1.0, levels, "abc"), ref)
        dA, dB, dC = sx.to_device(A), sx.to_device(B), sx.to_device(C)
        with pytest.raises(sx.StrassenError) as ei:
            sx.dgemm(dA, dB, dC, 1.0, 1.0, levels, "ab")
        assert ei.value.code == 2
        torch.cuda.synchronize()
        assert np.array_equal(sx.to_host(dC), C)
    finally:
        sx.set_workspace_limit(0)
    assert np.array_equal(run(A, B, C, 0.5, -1.5, levels, "ab"), free)


@pytest.mark.parametrize("shape,limits", [((4096, 4096, 4096), (100 << 20, 10 << 20)),
                                          ((4095, 4100, 4090), (600 << 20, 300 << 20))])
def test_staging_one_outer_product_at_a_time(shape, limits):
    """Two-level ABC where staging applies (in place, and on block-padded copies): a workspace
    cap that holds one outer product's sums but not all ten stages them product by product
    (ten sum passes instead of two), a smaller one forms them in the load (none); every form
    gives the same bits, and sampled columns match the oracle."""
    m, n, k = shape
    print(f"case staging one at a time {shape}", flush=True)
    A, B, C = W.problem(14, m, n, k, "uniform")
    dA, dB = sx.to_device(A), sx.to_device(B)

    def passes():
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            dC = sx.to_device(C)
            sx.dgemm(dA, dB, dC, 0.5, -1.25, 2, "abc")
            torch.cuda.synchronize()
        finally:
            sx.timing_enable(False)
        return sx.to_host(dC), sx.timing_collect("outer_sums")[1]

    full, n_full = passes()
    assert n_full == 2
    outs = []
    try:
        for limit, want in zip(limits, (10, 0)):
            sx.set_workspace_limit(limit)
            got, n_sums = passes()
            assert n_sums == want, (limit, n_sums)
            outs.append(got)
    finally:
        sx.set_workspace_limit(0)
    for got in outs:
        assert np.array_equal(got, full)
    cols = np.array([0, 1, n // 2, n - 1])
    ref = oracle_dgemm(A, np.asfortranarray(B[:, cols]), np.asfortranarray(C[:, cols]), 0.5, -1.25)
    assert rel_fro(full[:, cols], ref) <= 1e-11


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_every_tile_config_bitwise_and_exact(cfg, levels):
    """Every tile configuration gives the oracle's exact integer result and, on reals, the
    same bits as the automatic choice (per-element arithmetic does not depend on the tile)."""
    m, n, k = 1100, 1030, 1210
    print(f"case tile cfg {cfg} L={levels}", flush=True)
    A, B, C = W.problem(9, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    Ar, Br, Cr = W.problem(10, m, n, k, "uniform")
    try:
        sx.set_tile_config(-1)
        auto = [run(Ar, Br, Cr, 1.0, 1.0, levels, v) for v in (VARIANTS if levels else ["abc"])]
        sx.set_tile_config(cfg)
        for i, v in enumerate(VARIANTS if levels else ["abc"]):
            assert np.array_equal(run(A, B, C, 1.0, 1.0, levels, v), ref), v
            assert np.array_equal(run(Ar, Br, Cr, 1.0, 1.0, levels, v), auto[i]), v
    finally:
        sx.set_tile_config(-1)


@pytest.mark.parametrize("shape,beta", [((8192, 8192, 8192), 1.5), ((8188, 8190, 8196), 0.0)])
def test_one_level_staged_on_the_classical_kernel(shape, beta):
    """One-level ABC where its products fill whole rounds of the GPU on the classical kernel
    (k/2 >= 4096; the second shape has odd quadrant extents and tile fringes): the five sums of
    each side staged (two passes), then seven classical launches adding each product to its C
    quadrants; with a workspace cap that holds one product's two sums, seven sum passes; below
    that, the all-products kernel (no workspace).  Every form and the all-products kernel
    forced by configuration 4 give the same bits; sampled columns match the oracle (beta = 0:
    C, filled with NaN, is not read)."""
    m, n, k = shape
    print(f"case one-level staged classical {shape} beta={beta}", flush=True)
    A, B, C = W.problem(31, m, n, k, "uniform")
    if beta == 0.0:
        C[:] = np.nan
    dA, dB = sx.to_device(A), sx.to_device(B)

    def counted():
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            dC = sx.to_device(C)
            sx.dgemm(dA, dB, dC, -0.75, beta, 1, "abc")
            torch.cuda.synchronize()
        finally:
            sx.timing_enable(False)
        return (sx.to_host(dC), sx.timing_collect("outer_sums")[1],
                sx.timing_collect("classical")[1], sx.timing_collect("all_products")[1])

    staged, n_sums, n_cls, n_ap = counted()
    assert (n_sums, n_cls, n_ap) == (2, 7, 0)
    mq, nq, kq = m // 2, n // 2, k // 2
    one = 8 * (-(-(mq * kq) // 32) * 32 + -(-(kq * nq) // 32) * 32)
    outs = []
    try:
        for limit, want in ((one + 4096, (5 + 5, 7, 0)), (one // 2, (0, 0, 1))):
            sx.set_workspace_limit(limit)
            got, *counts = counted()
            assert tuple(counts) == want, (limit, counts)
            outs.append(got)
        sx.set_workspace_limit(0)
        sx.set_tile_config(4)
        outs.append(counted()[0])
    finally:
        sx.set_workspace_limit(0)
        sx.set_tile_config(-1)
    for got in outs:
        assert np.array_equal(got, staged)
    cols = np.array([0, 1, n // 2 - 1, n // 2, n - 1])
    Cc = np.asfortranarray(C[:, cols]) if beta != 0.0 else np.zeros((m, len(cols)), order="F")
    ref = oracle_dgemm(A, np.asfortranarray(B[:, cols]), Cc, -0.75, beta)
    assert rel_fro(staged[:, cols], ref) <= TOL[1]


def test_one_level_staged_on_the_classical_kernel_exact_on_integers():
    m, n, k = 8192, 8190, 8196
    print(f"case one-level staged classical integers {m}x{n}x{k}", flush=True)
    A, B, C = W.problem(32, m, n, k, "integer")
    got = run(A, B, C, 1.0, 1.0, 1, "abc")
    cols = np.array([0, 7, n // 2 - 1, n // 2, n - 1])
    ref = oracle_dgemm(A, np.asfortranarray(B[:, cols]), np.asfortranarray(C[:, cols]), 1.0, 1.0)
    assert np.array_equal(got[:, cols], ref)


# Shapes on which ABC runs the all-products kernel (m and k multiples of 2^(L+1)): full tiles,
# tile fringes inside the sub-blocks (m/4 = 194 = 3*64 + 2) and ragged n at both levels, and
# sub-blocks of whole k steps with ragged m and n (1000 x 1096 x 1024).
ALL_PRODUCTS_SHAPES = [(512, 512, 512), (1024, 1030, 1032), (776, 333, 1048), (64, 9, 8),
                       (1000, 1096, 1024)]


@pytest.mark.parametrize("shape", ALL_PRODUCTS_SHAPES)
@pytest.mark.parametrize("levels", [1, 2])
def test_all_products_kernel(shape, levels):
    """ABC on the all-products kernel: exact on integers, within the Strassen tolerance on reals,
    bitwise equal to AB, Naive and every tile configuration of the general kernel."""
    m, n, k = shape
    print(f"case all-products {shape} L={levels}", flush=True)
    A, B, C = W.problem(21, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    Ar, Br, Cr = W.problem(22, m, n, k, "uniform")
    refr = oracle_dgemm(Ar, Br, Cr.copy(order="F"), -0.5, 2.5)
    try:
        sx.set_tile_config(4)
        assert np.array_equal(run(A, B, C, 1.0, 1.0, levels, "abc"), ref)
        fused = run(Ar, Br, Cr, -0.5, 2.5, levels, "abc")
        assert rel_fro(fused, refr) <= TOL[levels]
        for v in ("ab", "naive"):
            assert np.array_equal(run(Ar, Br, Cr, -0.5, 2.5, levels, v), fused), v
        for cfg in (0, 1, 2, 3):
            sx.set_tile_config(cfg)
            assert np.array_equal(run(Ar, Br, Cr, -0.5, 2.5, levels, "abc"), fused), cfg
        # beta = 0: C is write-only (NaN in C must not show)
        sx.set_tile_config(4)
        Cn = np.full_like(Cr, np.nan)
        out = run(Ar, Br, Cn, 1.0, 0.0, levels, "abc")
        assert np.isfinite(out).all()
        assert np.array_equal(out, run(Ar, Br, Cn, 1.0, 0.0, levels, "naive"))
    finally:
        sx.set_tile_config(-1)


STAGED_SHAPES = [(512, 512, 512), (1032, 1028, 1048), (2048, 2056, 1024), (1000, 1096, 1024)]


@pytest.mark.parametrize("shape", STAGED_SHAPES)
def test_two_level_staged_outer_sums(shape):
    """Two-level ABC with the outer operand sums staged (tile configuration 5): exact on
    integers, within the Strassen tolerance on reals, bitwise equal to the unstaged all-products
    path and to Naive, and C write-only when beta = 0."""
    m, n, k = shape
    print(f"case staged {shape}", flush=True)
    A, B, C = W.problem(31, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    Ar, Br, Cr = W.problem(32, m, n, k, "uniform")
    refr = oracle_dgemm(Ar, Br, Cr.copy(order="F"), 0.75, -1.5)
    try:
        sx.set_tile_config(4)
        unstaged = run(Ar, Br, Cr, 0.75, -1.5, 2, "abc")
        sx.set_tile_config(5)
        assert np.array_equal(run(A, B, C, 1.0, 1.0, 2, "abc"), ref)
        staged = run(Ar, Br, Cr, 0.75, -1.5, 2, "abc")
        assert rel_fro(staged, refr) <= TOL[2]
        assert np.array_equal(staged, unstaged)
        assert np.array_equal(staged, run(Ar, Br, Cr, 0.75, -1.5, 2, "naive"))
        Cn = np.full_like(Cr, np.nan)
        out = run(Ar, Br, Cn, 1.0, 0.0, 2, "abc")
        assert np.isfinite(out).all()
        sx.set_tile_config(4)
        assert np.array_equal(out, run(Ar, Br, Cn, 1.0, 0.0, 2, "abc"))
    finally:
        sx.set_tile_config(-1)


def test_two_level_staging_default_and_small_caller_workspace():
    """At 8192 the default two-level ABC stages the outer sums (workspace reported), bitwise
    as the unstaged path; a caller workspace too small for the staging buffers makes it form the
    sums in the load instead (same bits, no error)."""
    import torch
    n = 8192
    print("case staging default 8192", flush=True)
    need = sx.workspace_size(n, n, n, 2, "abc")
    assert need >= 10 * (n // 2) ** 2 * 8
    A = W.device_uniform(41, n, n)
    B = W.device_uniform(42, n, n)
    C0 = W.device_uniform(43, n, n)
    outs = {}
    try:
        for name, cfg, ws in (("default", -1, None), ("unstaged", 4, None),
                              ("small_ws", -1, torch.empty(1 << 20, dtype=torch.float64,
                                                           device="cuda"))):
            sx.set_tile_config(cfg)
            sx.set_workspace(ws)
            C = C0.clone()
            sx.dgemm(A, B, C, 1.0, 1.0, 2, "abc")
            torch.cuda.synchronize()
            outs[name] = C
            sx.set_workspace(None)
    finally:
        sx.set_workspace(None)
        sx.set_tile_config(-1)
    assert torch.equal(outs["default"], outs["unstaged"])
    assert torch.equal(outs["small_ws"], outs["unstaged"])
    # spot check against the oracle on a few columns
    cols = [0, 4097, 8191]
    Ah = np.asfortranarray(A.cpu().numpy())
    Bc = np.asfortranarray(B[:, cols].cpu().numpy())
    ref = oracle_dgemm(Ah, Bc, np.asfortranarray(C0[:, cols].cpu().numpy()), 1.0, 1.0)
    assert rel_fro(outs["default"][:, cols].cpu().numpy(), ref) <= TOL[2]


def test_kernel_timing_hooks():
    """The library's event pairs: one all-products launch at one level, seven plus two staged
    outer-sum passes at two levels (m = n = k = 4096), one classical-kernel launch for levels 0."""
    import torch
    n = 4096
    print("case timing hooks", flush=True)
    A, B, C = (W.device_uniform(s, n, n) for s in (51, 52, 53))
    for kind in sx.KERNEL_KINDS:
        sx.timing_collect(kind)
    sx.timing_enable(True)
    try:
        sx.dgemm(A, B, C, 1.0, 1.0, 1, "abc")
        sx.dgemm(A, B, C, 1.0, 1.0, 2, "abc")
        sx.dgemm(A, B, C, 1.0, 1.0, 0, "abc")
        torch.cuda.synchronize()
    finally:
        sx.timing_enable(False)
    ms_ap, n_ap = sx.timing_collect("all_products")
    ms_os, n_os = sx.timing_collect("outer_sums")
    ms_t, n_t = sx.timing_collect("tile")
    ms_c, n_c = sx.timing_collect("classical")
    assert (n_ap, n_os, n_t, n_c) == (8, 2, 0, 1)
    assert ms_ap > 0 and ms_os > 0 and ms_c > 0
    assert sx.timing_collect("all_products") == (0.0, 0)


# Block-padded ABC: shapes and layouts the all-products kernel cannot take as given (odd and
# not-multiple-of-2^(L+1) m and k, odd leading dimensions, an operand one double off 16-byte
# alignment, two-level staging with n not a multiple of 4).
PADDED_CASES = [
    # (m, n, k, levels, lda_extra, ldb_extra, ldc_extra, offset, tile config)
    (301, 259, 271, 1, 0, 0, 0, 0, -1),
    (301, 259, 271, 2, 0, 0, 0, 0, -1),
    (1002, 998, 1030, 1, 0, 0, 0, 0, -1),      # m, k even, sub-block extents odd
    (1002, 998, 1030, 2, 0, 0, 0, 0, -1),
    (512, 512, 512, 1, 1, 3, 1, 0, -1),        # odd leading dimensions
    (512, 520, 512, 2, 0, 0, 0, 1, -1),        # every operand one double off alignment
    (1000, 1094, 1024, 2, 0, 0, 0, 0, 5),      # staged, n % 4 == 2
    (1001, 1094, 1027, 2, 2, 0, 0, 1, 5),      # staged, everything ragged
]


@pytest.mark.parametrize("case", PADDED_CASES)
def test_block_padded_abc(case):
    """ABC on block-padded copies: the copies run (timing hooks), the result is bitwise that of
    the unpadded path (the general tile kernel, Naive, and AB on its padded store form), exact on
    integers, within tolerance on reals, C write-only with beta = 0, and a caller workspace too
    small for the copies gives the same result without them."""
    m, n, k, levels, ea, eb, ec, off, cfg = case
    print(f"case padded {case}", flush=True)
    lda, ldb, ldc = m + ea, k + eb, m + ec
    A, B, C = W.problem(41, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    Ar, Br, Cr = W.problem(42, m, n, k, "uniform")
    refr = oracle_dgemm(Ar, Br, Cr.copy(order="F"), 0.5, -1.5)
    try:
        sx.set_tile_config(cfg)
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            got = run(Ar, Br, Cr, 0.5, -1.5, levels, "abc", lda, ldb, ldc, off)
        finally:
            sx.timing_enable(False)
        _, n_pad = sx.timing_collect("pad")
        _, n_ap = sx.timing_collect("all_products")
        assert n_pad >= 2 and n_ap >= 1, (n_pad, n_ap)
        assert rel_fro(got, refr) <= TOL[levels]
        assert np.array_equal(run(A, B, C, 1.0, 1.0, levels, "abc", lda, ldb, ldc, off), ref)
        Cn = np.full_like(Cr, np.nan)
        out0 = run(Ar, Br, Cn, 0.5, 0.0, levels, "abc", lda, ldb, ldc, off)
        assert np.isfinite(out0).all()
        sx.set_tile_config(0)   # the general tile kernel, unpadded
        assert np.array_equal(run(Ar, Br, Cr, 0.5, -1.5, levels, "abc", lda, ldb, ldc, off), got)
        assert np.array_equal(run(Ar, Br, Cn, 0.5, 0.0, levels, "abc", lda, ldb, ldc, off), out0)
        sx.set_tile_config(-1)
        assert np.array_equal(run(Ar, Br, Cr, 0.5, -1.5, levels, "naive", lda, ldb, ldc, off), got)
        # AB: the store form of the all-products kernel on padded A and B (one level, or two
        # with the staged outer sums; forced, as these problems are below the size from which
        # the default takes it), bitwise the products of the tile kernel
        sx.set_tile_config(4 if levels == 1 else 5)
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            got_ab = run(Ar, Br, Cr, 0.5, -1.5, levels, "ab", lda, ldb, ldc, off)
        finally:
            sx.timing_enable(False)
        n_ap_ab = sx.timing_collect("all_products")[1]
        assert n_ap_ab >= 1, n_ap_ab
        assert np.array_equal(got_ab, got)
        assert np.array_equal(run(A, B, C, 1.0, 1.0, levels, "ab", lda, ldb, ldc, off), ref)
    finally:
        sx.set_tile_config(-1)
    # a caller workspace too small for the copies: the unpadded path, the same result
    tiny = torch.empty(32, dtype=torch.float64, device="cuda")
    sx.set_workspace(tiny)
    try:
        sx.set_tile_config(cfg)
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            again = run(Ar, Br, Cr, 0.5, -1.5, levels, "abc", lda, ldb, ldc, off)
        finally:
            sx.timing_enable(False)
        assert sx.timing_collect("pad")[1] == 0
        assert np.array_equal(again, got)
    finally:
        sx.set_tile_config(-1)
        sx.set_workspace(None)


def test_ab_padded_by_default_from_192_positions():
    """AB by default: ragged problems with at least 192 tile positions of 64 x 64 per launch run
    the store form on block-padded A and B, smaller ones the tile kernel; both give the bits of
    ABC, within tolerance of the oracle and exact on integers."""
    for (m, n, k), fused in [((3001, 2777, 1333), True), ((1001, 777, 333), False)]:
        print(f"case ab default padded {(m, n, k)}", flush=True)
        A, B, C = W.problem(43, m, n, k, "uniform")
        ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
        Ai, Bi, Ci = W.problem(44, m, n, k, "integer")
        refi = oracle_dgemm(Ai, Bi, Ci.copy(order="F"), 1.0, 1.0)
        for kind in sx.KERNEL_KINDS:
            sx.timing_collect(kind)
        sx.timing_enable(True)
        try:
            got = run(A, B, C, 1.0, 1.0, 1, "ab")
        finally:
            sx.timing_enable(False)
        assert (sx.timing_collect("all_products")[1] >= 1) == fused
        assert (sx.timing_collect("pad")[1] >= 2) == fused
        assert rel_fro(got, ref) <= TOL[1]
        assert np.array_equal(got, run(A, B, C, 1.0, 1.0, 1, "abc"))
        assert np.array_equal(run(Ai, Bi, Ci, 1.0, 1.0, 1, "ab"), refi)


def test_probe_rates():
    """The matrix-core rate probe: FP64 and BF16 issue rates between half and 105% of the
    datasheet peaks (78.6 and 2500 TFLOP/s)."""
    print("case rate probe", flush=True)
    f64, bf16 = sx.probe_rates()
    print(f"  FP64 {f64:.2f} TFLOP/s, BF16 {bf16:.1f} TFLOP/s", flush=True)
    assert 0.5 * 78.6 < f64 < 1.05 * 78.6
    assert 0.5 * 2500.0 < bf16 < 1.05 * 2500.0


@pytest.mark.parametrize("shape,offset,kind", [
    ((4096, 4096, 528), 0, "integer"),    # whole tiles
    ((4094, 4093, 530), 0, "uniform"),    # ragged tiles (masked loads and stores)
    ((4097, 4096, 531), 0, "uniform"),    # m, k odd: block-padded copies
    ((4096, 4096, 520), 1, "uniform"),    # operands not 16-byte aligned: copies
])
def test_classical_kernel_bitwise_with_tile_kernel(shape, offset, kind):
    """The classical kernel on the fused load path (levels 0, default) performs the same FP64
    operations as the general tile kernel (forced with tile configuration 0): bitwise equal
    results; on integers both equal the oracle."""
    m, n, k = shape
    print(f"case classical kernel {shape} offset={offset} {kind}", flush=True)
    A, B, C = W.problem(81, m, n, k, kind)
    sx.timing_enable(True)
    try:
        sx.timing_collect("classical")
        got = run(A, B, C, 1.5, -0.5, 0, "abc", offset=offset)
        ms, launches = sx.timing_collect("classical")
        assert launches == 1
        sx.set_tile_config(0)
        try:
            ref = run(A, B, C, 1.5, -0.5, 0, "abc", offset=offset)
        finally:
            sx.set_tile_config(-1)
        assert sx.timing_collect("classical")[1] == 0
    finally:
        sx.timing_enable(False)
    assert np.array_equal(got, ref)
    if kind == "integer":
        assert np.array_equal(got, oracle_dgemm(A, B, C.copy(order="F"), 1.5, -0.5))
    else:
        assert (np.abs(got - oracle_dgemm(A, B, C.copy(order="F"), 1.5, -0.5))
                <= classical_bound(A, B, C, 1.5, -0.5)).all()


@pytest.mark.parametrize("levels,n", [(1, 8192), (2, 16384)])
def test_naive_on_classical_kernel_bitwise(levels, n):
    """Naive's products run on the classical kernel where the partition is exact and the products
    fill the CUs (timing hook: 7^L classical launches); the result stays bitwise that of ABC."""
    print(f"case naive on classical L={levels} n={n}", flush=True)
    A, B, C0 = (W.device_uniform(s, n, n) for s in (161, 162, 163))
    outs = {}
    sx.timing_enable(True)
    try:
        for k_ in sx.KERNEL_KINDS:
            sx.timing_collect(k_)
        for variant in ("naive", "abc"):
            C = C0.clone()
            sx.dgemm(A, B, C, 1.0, -1.0, levels, variant)
            torch.cuda.synchronize()
            outs[variant] = C
            if variant == "naive":
                assert sx.timing_collect("classical")[1] == 7 ** levels
                assert sx.timing_collect("tile")[1] == 0
    finally:
        sx.timing_enable(False)
    assert torch.equal(outs["naive"], outs["abc"])

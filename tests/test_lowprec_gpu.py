"""Reduced-precision mode on the GPU (BF16 / bf16x3 products on MFMA with FP32 accumulation)
against the CPU oracle of the same mode (oracle/lowprec.py) and the FP64 oracle.

  * small-integer inputs: every step is exact, so every mode must return the exact product
    (bit-exact against the FP64 oracle);
  * real inputs: |C_gpu - C_mode_oracle| <= the oracle's elementwise bound, which allows for
    FP32 accumulation in any order and the fused multiply-add of the update;
  * the operands themselves (sums and bf16 rounding) must be identical on both sides:
    test_operand_pass_bitwise reads the GPU's hi / lo operands back from a caller workspace and
    compares them bit for bit with the oracle's (the bound alone would let a truncating split
    or sums in the wrong precision through; tests/test_oracle_lowprec.py measures which
    planted mistakes each check catches).
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, rel_fro
from oracle.lowprec import gemm_lowprec

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
MODES = [(c, s, u) for c in ("bf16", "bf16x3") for s in ("f32", "f64") for u in ("f32", "f64")]


def run_ex(A, B, C, alpha, beta, levels, mode):
    compute, sp, cp = mode
    dA, dB, dC = sx.to_device(A), sx.to_device(B), sx.to_device(C)
    sx.gemm_ex(dA, dB, dC, alpha, beta, levels, compute, sp, cp)
    torch.cuda.synchronize()
    return sx.to_host(dC)


@pytest.mark.parametrize("shape", [(512, 512, 512), (300, 260, 270), (130, 70, 200)])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_integer_inputs_bit_exact(shape, levels):
    m, n, k = shape
    print(f"case lowprec integer {shape} L={levels}", flush=True)
    A, B, C = W.problem(41, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    for mode in MODES:
        assert np.array_equal(run_ex(A, B, C, 1.0, 1.0, levels, mode), ref), mode


@pytest.mark.parametrize("shape,kind", [((256, 256, 256), "uniform"), ((300, 260, 270), "uniform"),
                                        ((256, 192, 320), "wide_both")])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_real_inputs_within_bound(shape, kind, levels):
    m, n, k = shape
    print(f"case lowprec reals {shape} {kind} L={levels}", flush=True)
    A, B, C = W.problem(42, m, n, k, kind)
    for mode in MODES:
        ref, bound = gemm_lowprec(A, B, C, -0.5, 2.5, levels, *mode)
        got = run_ex(A, B, C, -0.5, 2.5, levels, mode)
        excess = np.abs(got - ref) - bound
        assert (excess <= 0).all(), (mode, float(excess.max()), float(np.abs(got - ref).max()))


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_beta_zero_nan_and_error_order(levels):
    m = n = k = 256
    print(f"case lowprec beta0 L={levels}", flush=True)
    A, B, C = W.problem(43, m, n, k, "uniform")
    Cn = np.full_like(C, np.nan)
    exact = oracle_dgemm(A, B, np.zeros_like(C, order="F"), 1.0, 0.0)
    err = {}
    for mode in (("bf16", "f64", "f64"), ("bf16x3", "f64", "f64")):
        got = run_ex(A, B, Cn, 1.0, 0.0, levels, mode)
        assert np.isfinite(got).all()
        err[mode[0]] = rel_fro(got, exact)
    assert err["bf16"] < 3e-2 and err["bf16x3"] < 1e-4 and err["bf16x3"] < 0.05 * err["bf16"]


def test_two_level_operands_larger_than_2gib():
    """Two-level bf16x3 operands of all 49 products exceed 2 GiB per side (m = k = 19200); every
    product's operand buffer is addressed from its own base.  Integer inputs: exact."""
    m, n, k = 19200, 128, 19200
    print(f"case lowprec large L=2 {m}x{n}x{k}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(44)
    A = torch.randint(-8, 9, (k, m), generator=g, device="cuda").to(torch.float64).t()
    B = torch.randint(-8, 9, (n, k), generator=g, device="cuda").to(torch.float64).t()
    C = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    assert sx.workspace_size_ex(m, n, k, 2, "bf16x3") > 2 ** 32
    sx.gemm_ex(A, B, C, 1.0, 0.0, 2, "bf16x3", "f64", "f64")
    torch.cuda.synchronize()
    cols = np.array([0, 17, 64, 127])
    A_h = sx.to_host(A)
    ref = oracle_dgemm(A_h, np.asfortranarray(sx.to_host(B)[:, cols]),
                       np.zeros((m, len(cols)), order="F"), 1.0, 0.0)
    got = C[:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_product_tile_widths_bitwise(levels, compute):
    """128 x 128 and 128 x 64 workgroup tiles of the product kernel (tile configuration 0 / 1)
    give the same bits: every C element sums the same k steps in the same order."""
    m, n, k = 520, 650, 390
    print(f"case tile widths L={levels} {compute}", flush=True)
    A, B, C = W.problem(91, m, n, k, "uniform")
    outs = []
    try:
        for cfg in (0, 1):
            sx.set_tile_config(cfg)
            dC = sx.to_device(C)
            sx.gemm_ex(sx.to_device(A), sx.to_device(B), dC, 0.75, -0.5, levels, compute, "f64", "f32")
            torch.cuda.synchronize()
            outs.append(sx.to_host(dC))
    finally:
        sx.set_tile_config(-1)
    assert np.array_equal(outs[0], outs[1])


def _bf16_bits(x32):
    """Upper 16 bits of float32 values that are exact bf16 values."""
    return (np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("sum_prec", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["uniform", "wide_both"])
def test_operand_pass_bitwise(levels, sum_prec, kind):
    """The bf16 operands the GPU forms (hi and lo of every product's A-side and B-side sum) are
    read from a caller workspace in the layout strassen_workspace_size_ex documents and compared
    bit for bit with the oracle's operand_sum + split_hi_lo (round to nearest even), padding
    zero.  This pins what the result bound cannot see: a truncating split or sums in the wrong
    precision stay inside that bound (tests/test_oracle_lowprec.py)."""
    from oracle.lowprec import operand_sum, split_hi_lo
    from oracle.tables import table
    m, n, k = 300, 260, 270
    print(f"case operand pass L={levels} {sum_prec} {kind}", flush=True)
    A, B, C = W.problem(61, m, n, k, kind)
    q = 2 ** levels
    mq, nq, kq = -(-m // q), -(-n // q), -(-k // q)
    mp, np_, kp = -(-mq // 128) * 128, -(-nq // 128) * 128, -(-kq // 64) * 64
    nprod = 7 ** levels
    need = sx.workspace_size_ex(m, n, k, levels, "bf16x3")
    assert need == 4 * nprod * (mp + np_) * kp
    ws = torch.full((need // 2 + 128,), -1, dtype=torch.int16, device="cuda")
    sx.set_workspace(ws)
    try:
        run_ex(A, B, C, 1.0, 1.0, levels, ("bf16x3", sum_prec, "f64"))
        raw = ws.cpu().numpy().view(np.uint16)
    finally:
        sx.set_workspace(None)
    sa, sb = mp * kp, np_ * kp
    TAh = raw[:nprod * sa].reshape(nprod, mp, kp)
    TBh = raw[nprod * sa:nprod * (sa + sb)].reshape(nprod, np_, kp)
    TAl = raw[nprod * (sa + sb):nprod * (2 * sa + sb)].reshape(nprod, mp, kp)
    TBl = raw[nprod * (2 * sa + sb):nprod * (2 * sa + 2 * sb)].reshape(nprod, np_, kp)
    for r, (a_t, b_t, _) in enumerate(table(levels)):
        ha, la = split_hi_lo(operand_sum(A, a_t, mq, kq, sum_prec))          # mq x kq
        hb, lb = split_hi_lo(operand_sum(B, b_t, kq, nq, sum_prec))          # kq x nq
        for got, want in ((TAh[r], _bf16_bits(ha)), (TAl[r], _bf16_bits(la)),
                          (TBh[r], _bf16_bits(hb.T)), (TBl[r], _bf16_bits(lb.T))):
            rows, cols = want.shape
            assert np.array_equal(got[:rows, :cols], want), r
            assert not got[rows:, :].any() and not got[:, cols:].any(), r   # zero padding

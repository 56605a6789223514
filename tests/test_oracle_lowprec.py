"""Pins of the reduced-precision oracle (oracle/lowprec.py) against things it does not compute
itself: torch's CPU bfloat16 conversion (round to nearest even), exact arithmetic on small
integers, the FP64 oracle, and the error behaviour of the hi/lo split."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, rel_fro
from oracle.lowprec import bf16_round, split_hi_lo, operand_sum, gemm_lowprec

torch = pytest.importorskip("torch")

MODES = [(c, s, u) for c in ("bf16", "bf16x3") for s in ("f32", "f64") for u in ("f32", "f64")]


def _torch_bf16(x32):
    return torch.from_numpy(x32.copy()).to(torch.bfloat16).to(torch.float32).numpy()


def test_bf16_round_matches_torch_conversion():
    g = np.random.default_rng(5)
    parts = [
        g.standard_normal(20000).astype(np.float32) * np.float32(1e3),
        (g.standard_normal(20000) * 1e-38).astype(np.float32),          # subnormal range
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, np.inf, -np.inf], dtype=np.float32),
    ]
    # exact ties: the low 16 bits are 0x8000, with even and odd kept parts
    base = g.integers(0x3F000000, 0x40000000, size=4000, dtype=np.uint32) & np.uint32(0xFFFF0000)
    parts.append((base | np.uint32(0x8000)).view(np.float32))
    x = np.concatenate(parts)
    assert np.array_equal(bf16_round(x), _torch_bf16(x))
    assert np.isnan(bf16_round(np.array([np.nan], dtype=np.float32))).all()


def test_split_hi_lo_properties():
    x = np.random.default_rng(6).uniform(-4, 4, 50000).astype(np.float32)
    hi, lo = split_hi_lo(x)
    assert np.array_equal(hi, _torch_bf16(x))
    assert np.array_equal(lo, _torch_bf16(x - hi))
    # hi + lo carries about 16 significant bits: |x - hi - lo| <= 2^-16 |x|
    r = np.abs(x.astype(np.float64) - hi - lo)
    assert (r <= 2.0 ** -16 * np.abs(x) + 1e-45).all()
    # hi alone: relative error <= 2^-8 (half an ulp of an 8-bit significand)
    assert (np.abs(x.astype(np.float64) - hi) <= 2.0 ** -8 * np.abs(x)).all()


def test_operand_sum_association_and_precision():
    """Two terms round once; four terms add the two pair sums; FP32 mode rounds every term
    to FP32 first.  Values chosen so that the other associations give other results."""
    big = 2.0 ** 30
    X = np.zeros((4, 4))
    # 4-term sum over blocks (0,0), (1,0), (0,1), (1,1) of a 2x2 partition (1x1 blocks)
    X[0, 0], X[1, 0], X[0, 1], X[1, 1] = big, 1.0, -big, 1.0
    terms = [((0, 0), 1), ((1, 0), 1), ((0, 1), 1), ((1, 1), 1)]
    # f64: (big + 1) + (-big + 1) = 2 exactly
    assert operand_sum(X[:2, :2], terms, 1, 1, "f64")[0, 0] == 2.0
    # f32: big + 1 rounds to big in FP32 (24-bit significand); pairs give big + (-big) = 0
    assert operand_sum(X[:2, :2], terms, 1, 1, "f32")[0, 0] == 0.0
    # sequential association would give ((big + 1) - big) + 1 = 2 in f64 and 1 in f32
    # sign factoring: -(x0 - x1) for the pair (-x0, +x1) when x0 == x1 gives -0.0
    Y = np.array([[1.5, 1.5]])
    v = operand_sum(Y, [((0, 0), -1), ((0, 1), 1)], 1, 1, "f64")[0, 0]
    assert v == 0.0 and np.signbit(v)


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("mode", MODES)
def test_integer_inputs_exact(levels, mode):
    """|entries| <= 8: every sum, bf16 operand and product is exact, so every mode gives the
    exact product (the FP64 oracle's result)."""
    compute, sp, cp = mode
    m, n, k = 70, 66, 84
    A, B, C = W.problem(31, m, n, k, "integer")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    out, bound = gemm_lowprec(A, B, C, 1.0, 1.0, levels, compute, sp, cp)
    assert np.array_equal(out, ref)
    # beta = 0 with NaN in C: C is not read
    out0, b0 = gemm_lowprec(A, B, np.full_like(C, np.nan), 2.0, 0.0, levels, compute, sp, cp)
    assert np.array_equal(out0, 2.0 * (A @ B))
    assert np.isfinite(b0).all()


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_real_inputs_error_ordering(levels):
    """On uniform reals: bf16x3 is far more accurate than bf16; both are close to the FP64
    result; the FP64 result itself is within its own bound."""
    m = n = k = 96
    A, B, C = W.problem(32, m, n, k, "uniform")
    ref = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    e = {}
    for compute in ("bf16", "bf16x3"):
        out, bound = gemm_lowprec(A, B, C, 1.0, 1.0, levels, compute, "f64", "f64")
        e[compute] = rel_fro(out, ref)
    assert e["bf16"] < 3e-2
    assert e["bf16x3"] < 1e-4
    assert e["bf16x3"] < 0.05 * e["bf16"]


def test_bound_is_positive_and_scales():
    A, B, C = W.problem(33, 40, 40, 40, "uniform")
    _, b1 = gemm_lowprec(A, B, C, 1.0, 1.0, 1, "bf16", "f32", "f32")
    _, b2 = gemm_lowprec(A, B, C, 2.0, 1.0, 1, "bf16", "f32", "f32")
    assert (b1 > 0).all() and (b2 >= b1).all()


# ---------------------------------------------------------------------------------------------
# Discriminating power of the two checks the GPU tests apply to the mode on real inputs:
#   (1) the operand pass: every bf16 hi / lo operand the GPU writes must equal, bit for bit,
#       the oracle's operand_sum + split_hi_lo (test_lowprec_gpu.py reads the GPU's operand
#       buffers from a caller workspace);
#   (2) the result: |C_gpu - C_oracle| <= gemm_lowprec's elementwise bound (FP32 accumulation
#       in any order is the one freedom the GPU has).
# A copy of the mode with one plausible mistake planted is run on the CPU; each mistake must
# be caught by at least one check, and the test records which one does.
# ---------------------------------------------------------------------------------------------
def _trunc_bf16(x):
    x = np.asarray(x, dtype=np.float32)
    return (x.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def _planted_operands(S, mistake):
    rnd = _trunc_bf16 if mistake == "trunc_all" else bf16_round
    hi = rnd(S)
    lo = (_trunc_bf16 if mistake in ("trunc_lo", "trunc_all") else bf16_round)(S - hi)
    return hi, lo


def _planted_mode(A, B, C, alpha, beta, levels, compute, sum_prec, mistake):
    """The mode of oracle/lowprec.py (FP64 C update) with `mistake` planted; returns the
    result and the operands of every product (hi, lo of both sides)."""
    from oracle.tables import table
    m, k = A.shape
    n = B.shape[1]
    q = 2 ** levels
    mq, nq, kq = -(-m // q), -(-n // q), -(-k // q)
    Cp = np.zeros((q * mq, q * nq))
    Cp[:m, :n] = C
    first = np.ones((q, q), dtype=bool)
    ops = []
    for a_t, b_t, c_t in table(levels):
        sp = "f64" if mistake == "f64_sums" else sum_prec
        ha, la = _planted_operands(operand_sum(A, a_t, mq, kq, sp), mistake)
        hb, lb = _planted_operands(operand_sum(B, b_t, kq, nq, sp), mistake)
        ops.append((ha, la, hb, lb))
        ha, la, hb, lb = (x.astype(np.float64) for x in (ha, la, hb, lb))
        M = ha @ hb
        if compute == "bf16x3":
            M = M + ha @ lb + (0.0 if mistake == "drop_cross" else la @ hb)
        for (ci, cj), gam in c_t:
            sl = (slice(ci * mq, (ci + 1) * mq), slice(cj * nq, (cj + 1) * nq))
            if first[ci, cj]:
                b = beta * beta if mistake == "beta_twice" else beta
                Cp[sl] = alpha * gam * M + b * Cp[sl]
            else:
                Cp[sl] = Cp[sl] + alpha * gam * M
            first[ci, cj] = False
    return Cp[:m, :n], ops


# (mistake, compute, sum_prec) -> caught by the bound?  (measured at 256^3, seed 42)
PLANTED = [
    ("trunc_lo", "bf16x3", "f64", False),     # truncating lo split: 0.03-0.25x the bound
    ("trunc_all", "bf16x3", "f64", False),    # truncating hi and lo: lo makes up for hi
    ("trunc_all", "bf16", "f64", True),       # truncating bf16: 77-440x
    ("drop_cross", "bf16x3", "f64", True),    # lo_A*hi_B dropped: 6-54x
    ("f64_sums", "bf16x3", "f32", False),     # FP64 sums where FP32 was asked
    ("beta_twice", "bf16x3", "f64", True),    # beta applied at two updates
    ("beta_twice", "bf16", "f32", True),
]


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("kind", ["uniform", "wide_both"])
@pytest.mark.parametrize("mistake,compute,sum_prec,by_bound", PLANTED)
def test_planted_mistakes_are_caught(mistake, compute, sum_prec, by_bound, levels, kind):
    A, B, C = W.problem(42, 256, 256, 256, kind)
    ref, bound = gemm_lowprec(A, B, C, -0.5, 2.5, levels, compute, sum_prec, "f64")
    got, ops = _planted_mode(A, B, C, -0.5, 2.5, levels, compute, sum_prec, mistake)
    _, clean = _planted_mode(A, B, C, -0.5, 2.5, levels, compute, sum_prec, "none")
    caught_bound = bool((np.abs(got - ref) > bound).any())
    if not (mistake == "f64_sums" and levels == 0):   # one term: FP64 and FP32 sums agree
        assert caught_bound == by_bound, (float(np.max(np.abs(got - ref) / bound)))
    used = [0, 2] if compute == "bf16" else [0, 1, 2, 3]
    caught_operands = any(not np.array_equal(o[i], c[i]) for o, c in zip(ops, clean) for i in used)
    assert caught_bound or caught_operands or (mistake == "f64_sums" and levels == 0)
    # the planted copy without a mistake is the oracle (same operands, result within rounding)
    assert np.allclose(_planted_mode(A, B, C, -0.5, 2.5, levels, compute, sum_prec, "none")[0],
                       ref, rtol=0, atol=1e-12)


def test_rne_and_truncation_differ_on_the_gpu_test_inputs():
    """The inputs of the GPU operand-pass test separate a round-to-nearest-even split from a
    truncating one in a large share of the lo parts."""
    A, _, _ = W.problem(61, 300, 260, 270, "uniform")
    S = operand_sum(A, [((0, 0), 1), ((1, 1), 1)], 150, 135, "f64")
    hi = bf16_round(S)
    lo_rne, lo_tr = bf16_round(S - hi), _trunc_bf16(S - hi)
    assert np.mean(lo_rne != lo_tr) > 0.3

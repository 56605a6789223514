"""Reduced-precision Strassen: the CPU reference for the BF16 / bf16x3 product mode.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The mode computes C := alpha*A*B + beta*C (A, B, C in FP64) with the products M_r of the
Strassen table (Sec. 3.1, Sec. 3.5) run on bf16 operands:

  1. operand sums  S = sum_s delta_s X_s  over the zero-padded sub-blocks, formed in FP64 or in
     FP32 (each term rounded to FP32 first); two terms are rounded once as c0*(x0 + (c0*c1)*x1),
     a four-term sum adds its two pair sums (the association of applying the one-level rule
     recursively); an FP64 sum is then rounded to FP32;
  2. bf16 operands: BF16 mode  hi = bf16(S);  bf16x3 mode  hi = bf16(S), lo = bf16(S - hi)
     (S - hi is exact in FP32); rounding to nearest, ties to even;
  3. products: BF16  M = hi_A hi_B;  bf16x3  M = hi_A hi_B + hi_A lo_B + lo_A hi_B; here the
     products of bf16 values are exact and the sums over k are done in FP64 (nearly exact);
  4. C update: for every C sub-block, in increasing product order, c := c + (alpha*gamma)*M_r,
     beta applied at the first update (beta = 0: C not read); in FP64, or in FP32 with C
     rounded to FP32 before its first update and every operation rounded to FP32.

The GPU accumulates M in FP32 and fuses the update's multiply and add; `gemm_lowprec` returns
with the result an elementwise bound on that difference, so a GPU result is
checked against it element by element.  On integer inputs small enough for every step to be
exact (|entries| <= 8, k <= 8192) the result is the exact product, whatever the mode.
"""
import numpy as np

from .tables import table

U32 = 2.0 ** -24
U64 = 2.0 ** -53


# ---------------------------------------------------------------------------------------------
# bf16 rounding and the hi/lo split
# ---------------------------------------------------------------------------------------------
def bf16_round(x):
    """Round float32 values to bf16 (8 significant bits), to nearest with ties to even.

    Returns float32 values that are exactly representable in bf16.  Works on the bit pattern:
    adding 0x7FFF plus the lowest kept bit to the 32-bit word and clearing the low 16 bits is
    round-to-nearest-even of the upper half (a carry into the exponent is the correct rounding
    up, up to infinity).  NaNs stay NaNs."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = np.where(nan, np.float32(np.nan), out)
    return out


def split_hi_lo(x32):
    """hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32."""
    x32 = np.asarray(x32, dtype=np.float32)
    hi = bf16_round(x32)
    lo = bf16_round(x32 - hi)
    return hi, lo


# ---------------------------------------------------------------------------------------------
# operand sums
# ---------------------------------------------------------------------------------------------
def _sub_block(X, bi, bj, rq, cq):
    """Sub-block (bi, bj) of the rq x cq partition of X, zero-padded to rq x cq."""
    out = np.zeros((rq, cq), dtype=np.float64)
    r0, c0 = bi * rq, bj * cq
    blk = X[r0:min(r0 + rq, X.shape[0]), c0:min(c0 + cq, X.shape[1])]
    out[:blk.shape[0], :blk.shape[1]] = blk
    return out


def operand_sum(X, terms, rq, cq, sum_prec):
    """The signed sum of `terms` (list of ((bi, bj), sign)) of X's sub-blocks as FP32 values."""
    dt = np.float64 if sum_prec == "f64" else np.float32
    xs = [_sub_block(X, b[0], b[1], rq, cq).astype(dt) for b, _ in terms]
    cs = [dt(s) for _, s in terms]

    def pair(i):
        c0, c1 = cs[i], cs[i + 1]
        return c0 * (xs[i] + (c0 * c1) * xs[i + 1])

    if len(terms) == 1:
        v = cs[0] * xs[0]
    elif len(terms) == 2:
        v = pair(0)
    elif len(terms) == 4:
        v = pair(0) + pair(2)
    else:
        raise ValueError("1, 2 or 4 terms")
    return np.asarray(v, dtype=np.float32)


# ---------------------------------------------------------------------------------------------
# the mode
# ---------------------------------------------------------------------------------------------
def _operands(S32, compute):
    hi = bf16_round(S32).astype(np.float64)
    if compute == "bf16":
        return hi, None
    lo = bf16_round(S32 - bf16_round(S32)).astype(np.float64)
    return hi, lo


def gemm_lowprec(A, B, C, alpha, beta, levels, compute="bf16", sum_prec="f32", c_prec="f64"):
    """Reduced-precision Strassen (the steps in the module docstring).

    Returns (C_out, bound): C_out the FP64 result, bound an elementwise bound on
    |C_gpu - C_out| for an implementation that accumulates M in FP32 and fuses the update."""
    if compute not in ("bf16", "bf16x3") or sum_prec not in ("f32", "f64") or \
            c_prec not in ("f32", "f64"):
        raise ValueError("mode")
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    C_in = np.asarray(C, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    q = 2 ** levels
    mq, nq, kq = -(-m // q), -(-n // q), -(-k // q)
    tab = table(levels)
    uc = U32 if c_prec == "f32" else U64

    # C in blocks (zero padded); c holds the running value in the update precision
    Cp = np.zeros((q * mq, q * nq))
    Cp[:m, :n] = C_in
    if c_prec == "f32":
        Cp = Cp.astype(np.float32).astype(np.float64)
    first = np.ones((q, q), dtype=bool)
    err_m = np.zeros((q * mq, q * nq))      # sum over updates of |alpha| * bound on M error
    upd = np.zeros((q * mq, q * nq))        # sum over updates of |c| + |alpha M|
    n_acc = kq if compute == "bf16" else 3 * kq
    g = n_acc * U32 / (1.0 - n_acc * U32)
    f32 = np.float32
    for a_terms, b_terms, c_terms in tab:
        SA = operand_sum(A, a_terms, mq, kq, sum_prec)
        SB = operand_sum(B, b_terms, kq, nq, sum_prec)
        ha, la = _operands(SA, compute)
        hb, lb = _operands(SB, compute)
        M = ha @ hb
        P = np.abs(ha) @ np.abs(hb)
        if compute == "bf16x3":
            M = M + ha @ lb + la @ hb
            P = P + np.abs(ha) @ np.abs(lb) + np.abs(la) @ np.abs(hb)
        for (ci, cj), gam in c_terms:
            sl = (slice(ci * mq, (ci + 1) * mq), slice(cj * nq, (cj + 1) * nq))
            c = Cp[sl]
            ag = alpha * gam
            if c_prec == "f64":
                if first[ci, cj]:
                    new = ag * M if beta == 0.0 else ag * M + beta * c
                else:
                    new = c + ag * M
            else:
                m32 = M.astype(f32)
                ag32, b32 = f32(ag), f32(beta)
                c32 = c.astype(f32)
                if first[ci, cj]:
                    new = ag32 * m32 if beta == 0.0 else ag32 * m32 + b32 * c32
                else:
                    new = c32 + ag32 * m32
                new = new.astype(np.float64)
            err_m[sl] += abs(alpha) * g * P
            prev = c if not first[ci, cj] else (beta * c if beta != 0.0 else 0.0 * M)
            upd[sl] += np.abs(prev) + abs(alpha) * np.abs(M)
            Cp[sl] = new
            first[ci, cj] = False
    out = Cp[:m, :n].copy()
    bound = (err_m + 3.0 * uc * upd + 4.0 * uc * np.abs(Cp))[:m, :n]
    return out, 2.0 * bound

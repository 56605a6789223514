"""The paper's performance model (Sec. 4.2, Fig. "tab:breakdown"), oracle side.

TEST INFRASTRUCTURE ONLY.  Evaluates T = T_a + T_m for BLAS dgemm and the one- and
two-level ABC / AB / Naive members, with the blocking parameters n_C, k_C and the
machine parameters tau_a (seconds per flop), tau_b (seconds per 8-byte word moved
from DRAM) and the prefetch efficiency lambda that scales the C-block row (*).

Readings (the paper is internally inconsistent for two levels):
  * `paper_counts=True` uses the coefficients exactly as printed
    (two-level T_a^{C+} = 154, N_m = 194/194/154, AB C+ = 462, Naive A+/B+ = 293).
  * `paper_counts=False` recounts them from the two-level table itself, by the
    rule that reproduces the printed one-level row: A/B reads = operand terms,
    ABC C-block reads/writes = C updates, AB/Naive temporaries = 3 words per
    C update plus the M writes, Naive sums = 2 words per term plus the writes.
"""
import math

VARIANTS = ("abc", "ab", "naive")

# N_m coefficients: (A_x, B_x, C_x, A_+, B_+, C_+)
_N_PAPER = {
    (0, "abc"): (1, 1, 1, 0, 0, 0),
    (1, "abc"): (12, 12, 12, 0, 0, 0),
    (1, "ab"): (12, 12, 7, 0, 0, 36),
    (1, "naive"): (7, 7, 7, 19, 19, 36),
    (2, "abc"): (194, 194, 154, 0, 0, 0),
    (2, "ab"): (194, 194, 49, 0, 0, 462),
    (2, "naive"): (49, 49, 49, 293, 293, 462),
}
_N_RECOUNT = dict(_N_PAPER)
_N_RECOUNT.update({
    (2, "abc"): (144, 144, 144, 0, 0, 0),
    (2, "ab"): (144, 144, 49, 0, 0, 432),
    (2, "naive"): (49, 49, 49, 193, 193, 432),
})
# extra additions: (products, A+ terms beyond one per product, B+ likewise, C+ updates)
_ADDS_PAPER = {0: (1, 0, 0, 0), 1: (7, 5, 5, 12), 2: (49, 95, 95, 154)}
_ADDS_RECOUNT = {0: (1, 0, 0, 0), 1: (7, 5, 5, 12), 2: (49, 95, 95, 144)}


def arithmetic_time(m, n, k, levels, tau_a, paper_counts=True):
    """T_a of the breakdown table (flops times tau_a)."""
    q = 2 ** levels
    prods, ap, bp, cp = (_ADDS_PAPER if paper_counts else _ADDS_RECOUNT)[levels]
    if levels == 0:
        return 2.0 * m * n * k * tau_a
    mq, nq, kq = m / q, n / q, k / q
    flops = prods * 2 * mq * nq * kq + ap * 2 * mq * kq + bp * 2 * kq * nq + cp * 2 * mq * nq
    return flops * tau_a


def memory_time(m, n, k, levels, variant, tau_b, n_c, k_c, lam=1.0, paper_counts=True):
    """T_m of the breakdown table; the C-block row is scaled by lam."""
    q = 2 ** levels
    variant = "abc" if levels == 0 else variant
    NAx, NBx, NCx, NAp, NBp, NCp = (_N_PAPER if paper_counts else _N_RECOUNT)[(levels, variant)]
    mq, nq, kq = m / q, n / q, k / q
    TAx = mq * kq * math.ceil(nq / n_c)
    TBx = nq * kq
    TCx = 2 * mq * nq * math.ceil(kq / k_c) * lam
    TAp = mq * kq
    TBp = nq * kq
    TCp = mq * nq
    words = NAx * TAx + NBx * TBx + NCx * TCx + NAp * TAp + NBp * TBp + NCp * TCp
    return words * tau_b


def total_time(m, n, k, levels, variant, tau_a, tau_b, n_c, k_c, lam=1.0, paper_counts=True):
    return (arithmetic_time(m, n, k, levels, tau_a, paper_counts)
            + memory_time(m, n, k, levels, variant, tau_b, n_c, k_c, lam, paper_counts))


def effective_gflops(m, n, k, seconds):
    """eq. (e:egflops1): 2mnk / time * 1e-9."""
    return 2.0 * m * n * k / seconds * 1e-9


# Machine of Sec. 5.1 (one core of the Xeon E5-2680 v2): 28.32 GFLOPS peak at
# 3.54 GHz, 59.7 GB/s over 4 channels, n_C = 4096, k_C = 256.  For one core
# tau_b is multiplied by the channel count (Sec. 4.2, "Notation").
IVY_ONE_CORE = dict(tau_a=1.0 / 28.32e9, tau_b=4 * 8.0 / 59.7e9, n_c=4096, k_c=256)


def predict_gflops(m, n, k, levels, variant, machine=IVY_ONE_CORE, lam=1.0, paper_counts=True):
    t = total_time(m, n, k, levels, variant, machine["tau_a"], machine["tau_b"],
                   machine["n_c"], machine["k_c"], lam, paper_counts)
    return effective_gflops(m, n, k, t)

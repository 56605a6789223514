"""Strassen operation tables, written from the paper (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A table lists, for every product M_r, the general operation of eq. (e:straprim4):
    M_r = (sum_s delta_s X_s)(sum_t eps_t V_t);   C_r' += gamma M_r  for each destination.
Each term is ((row_block, col_block), sign).  X_s are sub-blocks of A indexed
(i, p), V_t sub-blocks of B indexed (p, j), destinations sub-blocks of C (i, j).

ONE_LEVEL is Fig. "All operations for one-level Strassen" (Sec. 3.1) copied row
by row.  Tables for more levels follow Sec. 3.5: with the matrices split 2^L x 2^L,
product M_{7r+s} applies outer row r of the one-level table to the 2x2 grid of
2^(L-1)-blocks and inner row s of the (L-1)-level table inside them; block indices
combine as 2^(L-1)*outer + inner and coefficients multiply.  Terms are listed
inner-term-major (for each inner term, every outer term), the order in which the
paper prints the two-level table.  The paper's printed two-level operand sums lost
their minus signs; the composed signs are the reading used here (they satisfy the
matrix-multiplication identity, which the printed ones do not).
"""
import itertools

import numpy as np

P, M_ = +1, -1

# Fig. one-level (Sec. 3.1): (A terms, B terms, C updates)
ONE_LEVEL = [
    # M0 = (A00 + A11)(B00 + B11);  C00 += M0;  C11 += M0
    ([((0, 0), P), ((1, 1), P)], [((0, 0), P), ((1, 1), P)], [((0, 0), P), ((1, 1), P)]),
    # M1 = (A10 + A11) B00;  C10 += M1;  C11 -= M1
    ([((1, 0), P), ((1, 1), P)], [((0, 0), P)], [((1, 0), P), ((1, 1), M_)]),
    # M2 = A00 (B01 - B11);  C01 += M2;  C11 += M2
    ([((0, 0), P)], [((0, 1), P), ((1, 1), M_)], [((0, 1), P), ((1, 1), P)]),
    # M3 = A11 (B10 - B00);  C00 += M3;  C10 += M3
    ([((1, 1), P)], [((1, 0), P), ((0, 0), M_)], [((0, 0), P), ((1, 0), P)]),
    # M4 = (A00 + A01) B11;  C01 += M4;  C00 -= M4
    ([((0, 0), P), ((0, 1), P)], [((1, 1), P)], [((0, 1), P), ((0, 0), M_)]),
    # M5 = (A10 - A00)(B00 + B01);  C11 += M5
    ([((1, 0), P), ((0, 0), M_)], [((0, 0), P), ((0, 1), P)], [((1, 1), P)]),
    # M6 = (A01 - A11)(B10 + B11);  C00 += M6
    ([((0, 1), P), ((1, 1), M_)], [((1, 0), P), ((1, 1), P)], [((0, 0), P)]),
]

CLASSICAL = [([((0, 0), P)], [((0, 0), P)], [((0, 0), P)])]

# Winograd's variant (the Strassen-like scheme among the paper's references) in the general
# operation form: each product's operands flattened to signed sums of quadrants, and every
# C block it reaches.  With S1 = A10 + A11, S2 = S1 - A00, S3 = A00 - A10, S4 = A01 - S2,
# T1 = B01 - B00, T2 = B11 - T1, T3 = B11 - B01, T4 = T2 - B10, the products are
# M1 = A00 B00, M2 = A01 B10, M3 = S4 B11, M4 = A11 T4, M5 = S1 T1, M6 = S2 T2, M7 = S3 T3 and
# C00 = M1 + M2, C01 = M1 + M6 + M5 + M3, C10 = M1 + M6 + M7 - M4, C11 = M1 + M6 + M7 + M5.
WINOGRAD = [
    ([((0, 0), P)], [((0, 0), P)], [((0, 0), P), ((0, 1), P), ((1, 0), P), ((1, 1), P)]),
    ([((0, 1), P)], [((1, 0), P)], [((0, 0), P)]),
    ([((0, 1), P), ((1, 0), M_), ((1, 1), M_), ((0, 0), P)], [((1, 1), P)], [((0, 1), P)]),
    ([((1, 1), P)], [((1, 1), P), ((0, 1), M_), ((0, 0), P), ((1, 0), M_)], [((1, 0), M_)]),
    ([((1, 0), P), ((1, 1), P)], [((0, 1), P), ((0, 0), M_)], [((0, 1), P), ((1, 1), P)]),
    ([((1, 0), P), ((1, 1), P), ((0, 0), M_)], [((1, 1), P), ((0, 1), M_), ((0, 0), P)],
     [((0, 1), P), ((1, 0), P), ((1, 1), P)]),
    ([((0, 0), P), ((1, 0), M_)], [((1, 1), P), ((0, 1), M_)], [((1, 0), P), ((1, 1), P)]),
]


def winograd_table(levels):
    """Winograd's variant composed over `levels` levels (same rule as table())."""
    if levels == 0:
        return table(0)
    t = [tuple(list(x) for x in row) for row in WINOGRAD]
    for lev in range(2, levels + 1):
        q_in = 2 ** (lev - 1)
        inner = t
        t = []
        for (oa, ob, oc) in WINOGRAD:
            for (ia, ib, ic) in inner:
                t.append((_compose_terms(oa, ia, q_in), _compose_terms(ob, ib, q_in),
                          _compose_terms(oc, ic, q_in)))
    return t


def _compose_terms(outer, inner, q_in):
    out = []
    for (bi, si) in inner:
        for (bo, so) in outer:
            out.append(((q_in * bo[0] + bi[0], q_in * bo[1] + bi[1]), so * si))
    return out


def table(levels):
    """Operation table for `levels` levels (0 = one classical product)."""
    if levels < 0:
        raise ValueError("levels must be >= 0")
    if levels == 0:
        return [tuple(list(t) for t in row) for row in CLASSICAL]
    t = [tuple(list(x) for x in row) for row in ONE_LEVEL]
    for lev in range(2, levels + 1):
        q_in = 2 ** (lev - 1)
        inner = t
        t = []
        for (oa, ob, oc) in ONE_LEVEL:            # r: outer product
            for (ia, ib, ic) in inner:            # s: inner product -> index 7^(L-1) r + s
                t.append((_compose_terms(oa, ia, q_in),
                          _compose_terms(ob, ib, q_in),
                          _compose_terms(oc, ic, q_in)))
    return t


def coefficient_matrices(tab, levels):
    """Dense U (A), V (B), W (C) coefficient matrices, one row per product and
    one column per sub-block (row-major block index i*q + j)."""
    q = 2 ** levels
    R = len(tab)
    U = np.zeros((R, q * q), dtype=np.int64)
    V = np.zeros((R, q * q), dtype=np.int64)
    W = np.zeros((R, q * q), dtype=np.int64)
    for r, (a, b, c) in enumerate(tab):
        for (i, p), s in a:
            U[r, i * q + p] += s
        for (p, j), s in b:
            V[r, p * q + j] += s
        for (i, j), s in c:
            W[r, i * q + j] += s
    return U, V, W


def tensor_of(tab, levels):
    """Sum over products of U_r (x) V_r (x) W_r, a (q^2, q^2, q^2) integer array."""
    U, V, W = coefficient_matrices(tab, levels)
    return np.einsum("ra,rb,rc->abc", U, V, W)


def matmul_tensor(levels):
    """The block matrix-multiplication tensor: entry [(i,p), (p',j), (i',j')] is 1
    exactly when i = i', p = p', j = j' (Sec. 2.3, C_ij = sum_p A_ip B_pj)."""
    q = 2 ** levels
    T = np.zeros((q * q, q * q, q * q), dtype=np.int64)
    for i, p, j in itertools.product(range(q), repeat=3):
        T[i * q + p, p * q + j, i * q + j] = 1
    return T


def counts(tab):
    """(products, A terms, B terms, C updates)."""
    return (len(tab), sum(len(a) for a, _, _ in tab), sum(len(b) for _, b, _ in tab),
            sum(len(c) for _, _, c in tab))

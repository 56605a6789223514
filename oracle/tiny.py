"""Pure-Python loops for tiny sizes (oracle side, TEST INFRASTRUCTURE ONLY).

Matrices are lists of rows of Python floats/ints.
"""


def classical(A, B, C, alpha=1, beta=1):
    """C := alpha*A*B + beta*C by the definition of Sec. 2.1, sum in increasing p."""
    m, k, n = len(A), len(B), len(B[0]) if B else 0
    out = [[0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = 0
            for p in range(k):
                s = s + A[i][p] * B[p][j]
            out[i][j] = alpha * s + (beta * C[i][j] if beta != 0 else 0)
    return out


def block_2x2_eight_products(A, B):
    """A*B for 2x2 scalar matrices by the eight products of Sec. 2.3."""
    (a00, a01), (a10, a11) = A
    (b00, b01), (b10, b11) = B
    return [[a00 * b00 + a01 * b10, a00 * b01 + a01 * b11],
            [a10 * b00 + a11 * b10, a10 * b01 + a11 * b11]]


def strassen_2x2(A, B):
    """A*B for 2x2 scalar matrices by the seven products of Fig. one-level."""
    (a00, a01), (a10, a11) = A
    (b00, b01), (b10, b11) = B
    m0 = (a00 + a11) * (b00 + b11)
    m1 = (a10 + a11) * b00
    m2 = a00 * (b01 - b11)
    m3 = a11 * (b10 - b00)
    m4 = (a00 + a01) * b11
    m5 = (a10 - a00) * (b00 + b01)
    m6 = (a01 - a11) * (b10 + b11)
    c00 = m0 + m3 - m4 + m6
    c01 = m2 + m4
    c10 = m1 + m3
    c11 = m0 - m1 + m2 + m5
    return [[c00, c01], [c10, c11]]


def apply_table(tab, levels, A, B):
    """A*B for q x q scalar matrices (q = 2^levels) by executing a table literally:
    every product sums its operand terms, multiplies, and adds into its destinations."""
    q = 2 ** levels
    C = [[0] * q for _ in range(q)]
    for a_terms, b_terms, c_terms in tab:
        x = sum(s * A[i][p] for (i, p), s in a_terms)
        y = sum(s * B[p][j] for (p, j), s in b_terms)
        m = x * y
        for (i, j), s in c_terms:
            C[i][j] += s * m
    return C

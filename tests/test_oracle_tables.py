"""Pins for the oracle's operation tables (CPU only).

The one-level table is pinned by the exact matrix-multiplication tensor identity
and by the eight-product 2x2 definition of Sec. 2.3; the two-level table by the
same identity and by the term sets and C-update signs the paper prints in Fig.
"Computations for two-level Strassen".
"""
import copy
import itertools

import numpy as np
import pytest

from oracle import tables, tiny
from tests.conftest import read_golden


def _parse_signed(tok):
    return ((int(tok[1]), int(tok[2])), +1 if tok[0] == "+" else -1)


def test_one_level_matches_printed_figure():
    rows = read_golden("one_level_table.txt")
    assert len(rows) == 7
    for r, (idx, a, b, c) in enumerate(rows):
        assert int(idx) == r
        want = ([_parse_signed(t) for t in a.split()], [_parse_signed(t) for t in b.split()],
                [_parse_signed(t) for t in c.split()])
        got = tables.ONE_LEVEL[r]
        assert sorted(got[0]) == sorted(want[0])
        assert sorted(got[1]) == sorted(want[1])
        assert sorted(got[2]) == sorted(want[2])


@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_tensor_identity(levels):
    tab = tables.table(levels)
    assert np.array_equal(tables.tensor_of(tab, levels), tables.matmul_tensor(levels))


def test_counts():
    # Sec. 4.2: one level has 7 products and 5 extra additions on each operand;
    # two levels 49 products and 95 extra additions (144 terms - 49).
    assert tables.counts(tables.table(0)) == (1, 1, 1, 1)
    assert tables.counts(tables.table(1)) == (7, 12, 12, 12)
    assert tables.counts(tables.table(2)) == (49, 144, 144, 144)
    p, a, b, c = tables.counts(tables.table(2))
    assert a - p == 95 and b - p == 95
    p1, a1, b1, c1 = tables.counts(tables.table(1))
    assert a1 - p1 == 5 and b1 - p1 == 5 and c1 == 12


def test_term_limits():
    # Sec. 3.5: at two levels every operation sums up to four sub-blocks of A and of B
    # and updates up to four sub-blocks of C; at one level up to two (eq. e:straprim1).
    for levels, lim in ((1, 2), (2, 4)):
        for a, b, c in tables.table(levels):
            assert 1 <= len(a) <= lim and 1 <= len(b) <= lim and 1 <= len(c) <= lim
            assert all(s in (-1, 1) for _, s in a + b + c)


def test_two_level_matches_printed_term_sets_and_c_signs():
    rows = read_golden("two_level_table_as_printed.txt")
    tab = tables.table(2)
    assert len(rows) == 49
    for r, (idx, a, b, c) in enumerate(rows):
        assert int(idx) == r
        pa = [(int(t[0]), int(t[1])) for t in a.split()]
        pb = [(int(t[0]), int(t[1])) for t in b.split()]
        pc = sorted(((int(t[0]), int(t[1])), +1 if t[2] == "+" else -1) for t in c.split())
        ga, gb, gc = tab[r]
        # same sub-blocks, listed in the same order as printed
        assert [blk for blk, _ in ga] == pa, r
        assert [blk for blk, _ in gb] == pb, r
        assert sorted(gc) == pc, r


def test_two_level_printed_operand_signs_are_garbled():
    """Read literally (every operand term '+'), the printed two-level table does not
    compute A*B; the composed signs do.  This is the reading recorded for it."""
    rows = read_golden("two_level_table_as_printed.txt")
    literal = []
    for idx, a, b, c in rows:
        literal.append(([((int(t[0]), int(t[1])), 1) for t in a.split()],
                        [((int(t[0]), int(t[1])), 1) for t in b.split()],
                        [((int(t[0]), int(t[1])), +1 if t[2] == "+" else -1) for t in c.split()]))
    assert not np.array_equal(tables.tensor_of(literal, 2), tables.matmul_tensor(2))
    minus_a = sum(any(s < 0 for _, s in a) for a, _, _ in tables.table(2))
    minus_b = sum(any(s < 0 for _, s in b) for _, b, _ in tables.table(2))
    assert minus_a == 24 and minus_b == 24


def test_two_by_two_seven_products_equal_eight_products():
    g = np.random.default_rng(1)
    for _ in range(200):
        A = g.integers(-50, 51, size=(2, 2)).tolist()
        B = g.integers(-50, 51, size=(2, 2)).tolist()
        assert tiny.strassen_2x2(A, B) == tiny.block_2x2_eight_products(A, B)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_apply_table_on_scalars(levels):
    q = 2 ** levels
    g = np.random.default_rng(levels)
    tab = tables.table(levels)
    for _ in range(5):
        A = g.integers(-9, 10, size=(q, q)).tolist()
        B = g.integers(-9, 10, size=(q, q)).tolist()
        Z = [[0] * q for _ in range(q)]
        assert tiny.apply_table(tab, levels, A, B) == tiny.classical(A, B, Z, 1, 0)


def test_planted_sign_error_is_caught():
    """A single flipped sign anywhere in the one-level table breaks the identity."""
    base = tables.ONE_LEVEL
    for r, part, t in itertools.product(range(7), range(3), range(2)):
        if t >= len(base[r][part]):
            continue
        bad = copy.deepcopy([list(map(list, row)) for row in base])
        blk, s = bad[r][part][t]
        bad[r][part][t] = (blk, -s)
        bad = [tuple(row) for row in bad]
        assert not np.array_equal(tables.tensor_of(bad, 1), tables.matmul_tensor(1))

"""Pins for the oracle's port of the paper's performance model (CPU only).

Pinned by the closed form printed for one level (Sec. 4.2, "Arithmetic
operations"), the coefficient table as printed (Fig. tab:breakdown), and the
qualitative predictions of Sec. 4.3 ("Discussion").
"""
import pytest

from oracle import costmodel as cm
from tests.conftest import read_golden

IVY = cm.IVY_ONE_CORE


def test_coefficients_as_printed():
    rows = read_golden("breakdown_coefficients.txt")
    for head, vals in rows:
        name, lev = head.split()
        v = tuple(int(x) for x in vals.split())
        if name == "arith":
            assert cm._ADDS_PAPER[int(lev)] == v
        else:
            key = (int(lev), "abc" if name == "dgemm" else name)
            assert cm._N_PAPER[key] == v


@pytest.mark.parametrize("m,n,k", [(1000, 1000, 1000), (16000, 16000, 512), (300, 700, 50)])
def test_one_level_arithmetic_closed_form(m, n, k):
    ta = cm.arithmetic_time(m, n, k, 1, 1.0)
    assert ta == pytest.approx(1.75 * m * n * k + 2.5 * m * k + 2.5 * k * n + 6 * m * n, rel=1e-12)


def test_two_level_recount_matches_table_terms():
    from oracle import tables
    p, a, b, c = tables.counts(tables.table(2))
    assert cm._ADDS_RECOUNT[2] == (p, a - p, b - p, c)
    assert cm._N_RECOUNT[(2, "abc")][:3] == (a, b, c)


def g(m, n, k, L, v):
    return cm.predict_gflops(m, n, k, L, v, IVY)


def test_asymptotic_order():
    # large problems: two-level > one-level > dgemm
    n = 16000
    assert g(n, n, n, 2, "ab") > g(n, n, n, 1, "ab") > g(n, n, n, 0, "abc")


def test_abc_vs_ab_square():
    # ABC wins for small squares, AB for large ones, at one and two levels
    for L in (1, 2):
        assert g(1000, 1000, 1000, L, "abc") > g(1000, 1000, 1000, L, "ab")
        assert g(16000, 16000, 16000, L, "ab") > g(16000, 16000, 16000, L, "abc")


def test_rank_k_abc_peak_at_multiple_of_kc():
    m = n = 16000
    kc = IVY["k_c"]
    # k = 2 k_C (one level), 4 k_C (two levels): ABC is the best member
    assert g(m, n, 2 * kc, 1, "abc") > max(g(m, n, 2 * kc, 1, "ab"), g(m, n, 2 * kc, 1, "naive"),
                                           g(m, n, 2 * kc, 0, "abc"))
    assert g(m, n, 4 * kc, 2, "abc") > max(g(m, n, 4 * kc, 2, "ab"), g(m, n, 4 * kc, 2, "naive"))


def test_switch_point_near_500_for_abc():
    # Sec. 3.3 reports a switch point as small as 500 (one core); the model puts
    # one-level ABC ahead of dgemm already at 1000 and behind at 100.
    assert g(1000, 1000, 1000, 1, "abc") > g(1000, 1000, 1000, 0, "abc")
    assert g(100, 100, 100, 1, "abc") < g(100, 100, 100, 0, "abc") * 1.001

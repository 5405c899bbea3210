"""The per-DOF FLOP counts that bench.py divides by kernel time (roofline
"achieved"): the Sec. 3.6 lower bound and its extension to m != n points.
CPU only."""
import itertools
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _sumfact_fmas(n, m, d=3):
    """Multiply-adds of one sum factorization from n^d coefficients to m^d
    points, counted by walking its loops (Sec. 3.2): direction q maps
    (m^(q-1) n^(d-q+1)) entries to (m^q n^(d-q)), n multiply-adds per output."""
    count = 0
    shape = [n] * d
    for q in range(d):
        shape[q] = m
        for _ in itertools.product(*[range(s) for s in shape]):
            count += n
    return count


def test_sum_factorization_cost_matches_loop_count():
    # Cost_vol = 2 C m^(d+1) FLOP with C = sum_q (n/m)^q, one FMA = 2 FLOP
    for n, m in [(2, 2), (2, 4), (3, 5), (4, 4), (4, 6), (5, 7)]:
        C = sum((n / m) ** q for q in range(1, 4))
        assert abs(_sumfact_fmas(n, m) - C * m ** 4) < 1e-9


def test_rectangular_count_reduces_to_the_paper_formula():
    for k in range(1, 11):
        assert abs(bench.flop_per_dof_rect(k, k + 1) - bench.flop_per_dof(k)) < 1e-9
    # the printed formula at d = 3, p = 7: 4*4*3*8 + 18 + 15 + 3 + 8*4*9 + 3*(18+24+18)/8
    assert abs(bench.flop_per_dof(7) - (384 + 36 + 288 + 22.5)) < 1e-12


def test_rectangular_count_grows_with_the_points():
    for k in range(1, 9):
        a, b = bench.flop_per_dof_rect(k, k + 1), bench.flop_per_dof_rect(k, k + 3)
        assert b > a
    # k = 1, m = 4 by hand: C = 7/8; volume (16 C 4^4 + 36 * 4^3) / 8 = 736,
    # faces (96 C 4^3 + 180 * 4^2) / 8 = 1032
    assert abs(bench.flop_per_dof_rect(1, 4) - 1768.0) < 1e-9

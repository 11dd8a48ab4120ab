"""Pins for the exact tier of the oracle (oracle/racah.py).

The Racah sum is checked against things that do not share its formula:
sympy's independent Wigner-3j routine, the textbook closed form for the
(0 0 0) symbol (E57 eq. 3.7.17), the closed forms for l3 = 0 and l3 = 1,
the orthogonality sums, and the permutation / m-flip symmetries of Sec. 3
(eqs. permutation, mflip).
"""
import itertools
import math
from fractions import Fraction

import pytest
import sympy
from sympy.physics.wigner import wigner_3j

from oracle import racah


def _sympy_sq_sign(j1, j2, j3, m1, m2, m3):
    v = wigner_3j(j1, j2, j3, m1, m2, m3)
    if v == 0:
        return 0, Fraction(0)
    sq = sympy.Rational(v ** 2)
    return int(sympy.sign(v)), Fraction(int(sq.p), int(sq.q))


def test_racah_equals_sympy_small():
    n = 0
    for j1, j2 in itertools.product(range(0, 7), repeat=2):
        for j3 in range(abs(j1 - j2), j1 + j2 + 1):
            for m1 in range(-min(j1, 2), min(j1, 2) + 1):
                for m2 in range(-min(j2, 2), min(j2, 2) + 1):
                    m3 = -m1 - m2
                    if abs(m3) > j3:
                        continue
                    assert racah.threej_sq_sign(j1, j2, j3, m1, m2, m3) == \
                        _sympy_sq_sign(j1, j2, j3, m1, m2, m3), (j1, j2, j3, m1, m2, m3)
                    n += 1
    assert n > 1000


@pytest.mark.parametrize("l1,l2,l3,m", [(17, 23, 30, -2), (40, 41, 9, -2), (25, 25, 50, 0),
                                        (33, 12, 31, -2), (60, 70, 90, -2)])
def test_racah_equals_sympy_medium(l1, l2, l3, m):
    assert racah.threej_sq_sign(l1, l2, l3, m, -m, 0) == _sympy_sq_sign(l1, l2, l3, m, -m, 0)


def _closed_form_000(j1, j2, j3):
    """E57 eq. 3.7.17: for J = 2g even,
    (j1 j2 j3; 0 0 0) = (-1)^g sqrt[(2g-2j1)!(2g-2j2)!(2g-2j3)!/(2g+1)!]
                        * g! / [(g-j1)!(g-j2)!(g-j3)!],  and 0 for odd J."""
    J = j1 + j2 + j3
    if J % 2 or j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0, Fraction(0)
    g = J // 2
    f = math.factorial
    sq = Fraction(f(2 * g - 2 * j1) * f(2 * g - 2 * j2) * f(2 * g - 2 * j3), f(2 * g + 1)) \
        * Fraction(f(g), f(g - j1) * f(g - j2) * f(g - j3)) ** 2
    return (-1 if g % 2 else 1), sq


def test_racah_000_equals_closed_form():
    for j1, j2 in itertools.product(range(0, 31, 3), range(0, 31, 2)):
        for j3 in range(abs(j1 - j2), j1 + j2 + 1):
            assert racah.threej_sq_sign(j1, j2, j3, 0, 0, 0) == _closed_form_000(j1, j2, j3)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 7, 20, 45])
def test_racah_l3_zero_and_one(l):
    # (l l 0; m -m 0) = (-1)^(l-m)/sqrt(2l+1);  (l l 1; m -m 0) = (-1)^(l-m) m/sqrt(l(l+1)(2l+1))
    for m in range(-l, l + 1):
        sg, sq = racah.threej_sq_sign(l, l, 0, m, -m, 0)
        assert sq == Fraction(1, 2 * l + 1)
        assert sg == (-1) ** ((l - m) % 2)
        if l >= 1:
            sg, sq = racah.threej_sq_sign(l, l, 1, m, -m, 0)
            assert sq == Fraction(m * m, l * (l + 1) * (2 * l + 1))
            if m != 0:
                assert sg == (-1) ** ((l - m) % 2) * (1 if m > 0 else -1)


@pytest.mark.parametrize("j1,j2", [(2, 2), (5, 3), (9, 14), (20, 20), (13, 2)])
@pytest.mark.parametrize("m", [0, -2, 1])
def test_racah_orthogonality(j1, j2, m):
    if abs(m) > min(j1, j2):
        pytest.skip("no such symbol")
    total = sum((2 * j3 + 1) * racah.threej_sq_sign(j1, j2, j3, m, -m, 0)[1]
                for j3 in range(abs(j1 - j2), j1 + j2 + 1))
    assert total == 1


@pytest.mark.parametrize("j1,j2", [(2, 2), (5, 3), (9, 14), (20, 20)])
def test_racah_cross_orthogonality(j1, j2):
    # sum_j3 (2j3+1)(j1 j2 j3; 0 0 0)(j1 j2 j3; -2 2 0) = 0 (different m1 at fixed m3)
    s = sum((2 * j3 + 1) * racah.threej_product(j1, j2, j3, racah.M000, racah.M220)
            for j3 in range(abs(j1 - j2), j1 + j2 + 1))
    assert abs(s) < Fraction(1, 2 ** 200)


def test_racah_symmetries():
    for (j1, j2, j3) in [(3, 4, 5), (6, 6, 2), (7, 3, 5), (10, 9, 12)]:
        for (m1, m2) in [(0, 0), (-2, 2), (1, -2), (2, 1)]:
            m3 = -m1 - m2
            if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
                continue
            base = racah.threej_sq_sign(j1, j2, j3, m1, m2, m3)
            J = j1 + j2 + j3
            ph = -1 if J % 2 else 1
            # even (cyclic) permutations leave the symbol unchanged
            assert racah.threej_sq_sign(j2, j3, j1, m2, m3, m1) == base
            assert racah.threej_sq_sign(j3, j1, j2, m3, m1, m2) == base
            # odd permutations and the m-flip multiply by (-1)^J
            assert racah.threej_sq_sign(j2, j1, j3, m2, m1, m3) == (ph * base[0], base[1])
            assert racah.threej_sq_sign(j1, j2, j3, -m1, -m2, -m3) == (ph * base[0], base[1])


def test_racah_selection_rules():
    assert racah.threej_sq_sign(3, 4, 8, 0, 0, 0) == (0, 0)      # outside the triangle
    assert racah.threej_sq_sign(3, 4, 6, 0, 0, 0) == (0, 0)      # odd J with all m = 0
    assert racah.threej_sq_sign(1, 4, 4, -2, 2, 0) == (0, 0)     # |m| > j
    assert racah.threej_sq_sign(3, 4, 5, 1, 1, 1) == (0, 0)      # m sum != 0
    assert racah.threej_sq_sign(3, 4, 6, -2, 2, 0)[0] != 0       # (-2 2 0) lives at odd J too

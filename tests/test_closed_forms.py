"""The per-term closed forms the strip kernels evaluate, checked exactly
against the Racah sum of the oracle's exact tier (rational arithmetic).

Even L (App. B.3, eq. 022_linear_closedform with (j1, j2, j3) = (l3, l1, l2)
and the (0 0 0) ratio from eq. 000_sq_main / eq. g_rec):
    (l1 l2 l3; -2 2 0) = (l1 l2 l3; 0 0 0) N' c_l1 c_l2 / 2,
    N' = c (c - 2(a+b-1)) + a(a-2) + b(b-2).
Odd L (eq. 022_rearranged with eq. joneodd and eq. joneevensimp at j3 + 1):
    (l1 l2 l3; -2 2 0)^2 = (l1, l2+1, l3; 0 0 0)^2 (c_l1 c_l2 / 2)^2
                           (sig(sig+1) - c)(c - d(d+1))(c + mu)^2,
    sig = l1 + l2 + 1, tau = sig + 1, mu = 2 (l1+2)(l2+2) - tau(tau+1), d = l2 - l1.
c_l^2 = 1/((l-1) l (l+1)(l+2)).  These are the formulas of the HIP kernels
restated, not oracle code; the oracle never uses them.
"""
from fractions import Fraction

import pytest

from oracle.racah import threej_sq_sign


def _cl2(l):
    return Fraction(1, (l - 1) * l * (l + 1) * (l + 2))


def _even_nprime(l1, l2, l3):
    a, b, c = l1 * (l1 + 1), l2 * (l2 + 1), l3 * (l3 + 1)
    return c * (c - 2 * (a + b - 1)) + a * (a - 2) + b * (b - 2)


def _odd_factor(l1, l2, l3):
    d, c = l2 - l1, l3 * (l3 + 1)
    sg = l1 + l2 + 1
    tau = sg + 1
    mu = 2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1)
    return (sg * (sg + 1) - c) * (c - d * (d + 1)) * (c + mu) ** 2


def _cases(lmax):
    for l1 in range(2, lmax + 1):
        for l2 in range(l1, lmax + 1):
            for l3 in range(l2 - l1, l1 + l2 + 1):
                yield l1, l2, l3


@pytest.mark.parametrize("lo,hi", [(2, 14), (40, 43)])
def test_even_l_collapsed_form(lo, hi):
    n = 0
    for l1 in range(lo, hi + 1):
        for l2 in range(l1, hi + 1):
            for l3 in range(l2 - l1, l1 + l2 + 1, 2):       # even L
                sz, z2 = threej_sq_sign(l1, l2, l3, -2, 2, 0)
                sx, x2 = threej_sq_sign(l1, l2, l3, 0, 0, 0)
                nprime = _even_nprime(l1, l2, l3)
                # squares agree, and the sign of Z is sign(X) sign(N')
                assert z2 == x2 * nprime ** 2 * _cl2(l1) * _cl2(l2) / 4
                if z2:
                    assert sz == sx * (1 if nprime > 0 else -1)
                n += 1
    assert n > 100


@pytest.mark.parametrize("lo,hi", [(2, 15), (37, 40)])
def test_odd_l_reduction(lo, hi):
    n = 0
    for l1 in range(lo, hi + 1):
        for l2 in range(l1, hi + 1):
            for l3 in range(l2 - l1 + 1, l1 + l2 + 1, 2):   # odd L
                _, z2 = threej_sq_sign(l1, l2, l3, -2, 2, 0)
                _, y2 = threej_sq_sign(l1, l2 + 1, l3, 0, 0, 0)
                assert z2 == y2 * _cl2(l1) * _cl2(l2) / 4 * _odd_factor(l1, l2, l3)
                n += 1
    assert n > 100


def test_odd_l_last_step_vanishes():
    """The strip walk of diagonal d+1 runs one step past l3 = l1 + l2 - 1; there
    the factor sig(sig+1) - c is exactly 0."""
    for l1 in range(2, 30):
        for l2 in range(l1, 30):
            assert _odd_factor(l1, l2, l1 + l2 + 1) == 0


def _spin1_even(l1, l2, l3):
    """(l1 l2 l3; -1 1 0)^2 / (0 0 0)^2 and the sign factor for even L:
    Z = -X (a + b - c) / (2 sqrt(ab))."""
    a, b, c = l1 * (l1 + 1), l2 * (l2 + 1), l3 * (l3 + 1)
    return Fraction((a + b - c) ** 2, 4 * a * b), -1 if a + b - c > 0 else (1 if a + b - c < 0 else 0)


@pytest.mark.parametrize("lo,hi", [(1, 15), (40, 43)])
def test_spin1_closed_forms(lo, hi):
    """The (-1 1 0) symbol as the threej kernel evaluates it: even L one
    product with (0 0 0); odd L eq. joneodd with (j1, j2, j3) = (l3, l1, l2),
    i.e. -1/2 [(L+2)(L-2 l3+1)(L-2 l1+1)(L-2 l2)/(ab)]^{1/2} (l1, l2+1, l3; 0 0 0)."""
    n = 0
    for l1 in range(lo, hi + 1):
        for l2 in range(lo, hi + 1):
            for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                L = l1 + l2 + l3
                sz, z2 = threej_sq_sign(l1, l2, l3, -1, 1, 0)
                a, b = l1 * (l1 + 1), l2 * (l2 + 1)
                if L % 2 == 0:
                    sx, x2 = threej_sq_sign(l1, l2, l3, 0, 0, 0)
                    r2, sg = _spin1_even(l1, l2, l3)
                    assert z2 == x2 * r2
                    if z2:
                        assert sz == sx * sg
                else:
                    sy, y2 = threej_sq_sign(l1, l2 + 1, l3, 0, 0, 0)
                    f2 = Fraction((L + 2) * (L - 2 * l3 + 1) * (L - 2 * l1 + 1) * (L - 2 * l2), 4 * a * b)
                    assert z2 == f2 * y2
                    if z2:
                        assert sz == -sy
                n += 1
    assert n > 100


@pytest.mark.parametrize("lo,hi", [(2, 15), (37, 40)])
def test_odd_l_sign(lo, hi):
    """Signed odd-L (-2 2 0): Z = -Y' (c + mu) (c_l1 c_l2 / 2) [(sig(sig+1) - c)(c - d(d+1))]^{1/2}."""
    for l1 in range(lo, hi + 1):
        for l2 in range(lo, hi + 1):
            for l3 in range(l2 - l1 + 1 if l2 >= l1 else l1 - l2 + 1, l1 + l2 + 1, 2):
                sz, z2 = threej_sq_sign(l1, l2, l3, -2, 2, 0)
                if not z2:
                    continue
                sy, _ = threej_sq_sign(l1, l2 + 1, l3, 0, 0, 0)
                c = l3 * (l3 + 1)
                tau = l1 + l2 + 2
                mu = 2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1)
                assert sz == -sy * (1 if c + mu > 0 else -1)

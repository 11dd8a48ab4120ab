"""The symbol families of the Conclusion, (1 1 -2) and (2 2 -4), and their
relatives (l1 l2 l3; m1 m2 m3) with small magnetic numbers (CPU only).

1. The oracle's general Schulten--Gordon rows (oracle_threej_row_m) against
   the Racah sum of the exact tier: every pair l1, l2 <= 12 for a set of
   magnetic numbers including sign flips and mixed signs, and sampled
   symbols of rows at l ~ 200-400.

2. The closed forms the couple_threej_rows_m kernel evaluates, checked
   exactly (rational squares and signs) against the Racah sum.  Every triple
   m1 + m2 + m3 = 0 is brought, by a cyclic permutation of the columns and
   at most one m-flip (a factor (-1)^L), to F_ab(x, y, z) = (x y z; a b -a-b)
   with a, b >= 0.  For 0 <= a, b <= 2:

       even L:  F_ab = X N_ab / (2 D_ab),    X = (x y z; 0 0 0),
       odd L:   F_ab = W N_ab / (2 D_ab),
                W^2 = (x, y, z+1; 0 0 0)^2 (L+2)(L+1-2x)(L+1-2y)(L-2z),
                sign W = (-1)^((L+1)/2),
       D_ab^2 = prod_{k<a} (A - k(k+1)) prod_{k<b} (B - k(k+1))
                prod_{k<a+b} (C - k(k+1)),
       A = x(x+1), B = y(y+1), C = z(z+1), s = A - B, t = A + B,

   with the integer polynomials N_ab below.  They come from the App. B
   closed forms of the (0 -1 1) and (0 -2 2) families (on the lines a = 0
   and b = 0) carried into the quadrant by the lowering relation of E57
   Sec. 3.7,
       sqrt((x+a)(x-a+1)) F_{a-1,b} + sqrt((y+b)(y-b+1)) F_{a,b-1}
         + sqrt((z+a+b)(z-a-b+1)) F_ab = 0,
   which is itself checked here.  W is also checked in its table form
   8 p1 p2 p3 (L+2) g(p1) g(p2) g(p3) / ((L+2) g(P')), P' = (L+1)/2,
   p_i = P' - l_i, the form the kernel reads from the g(p) tables.

These are the kernel's formulas restated, not oracle code; the oracle never
uses them.
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

from oracle.racah import threej, threej_sq_sign


def numerator(a, b, odd, A, B, C):
    """N_ab(A, B, C) of the family closed forms (exact integers)."""
    s, t = A - B, A + B
    table = {
        (0, 0, 0): lambda: 2,
        (0, 0, 1): lambda: 0,
        (0, 1, 0): lambda: s - C,
        (0, 1, 1): lambda: 1,
        (0, 2, 0): lambda: C * C - C * (t + s + 2) + s * s + 2 * s,
        (0, 2, 1): lambda: s - C + 2,
        (1, 0, 0): lambda: -(s + C),
        (1, 0, 1): lambda: -1,
        (1, 1, 0): lambda: C * t - s * s,
        (1, 1, 1): lambda: -s,
        (1, 2, 0): lambda: -C * C * A + C * ((s * s + 3 * s * t) // 2 + s + 3 * t) - s ** 3 - 3 * s * s - s * t,
        (1, 2, 1): lambda: C * A - s * s - 3 * s - t,
        (2, 0, 0): lambda: C * C - C * (t - s + 2) + s * s - 2 * s,
        (2, 0, 1): lambda: s + C - 2,
        (2, 1, 0): lambda: -C * C * B + C * ((s * s - 3 * s * t) // 2 - s + 3 * t) + s ** 3 - 3 * s * s + s * t,
        (2, 1, 1): lambda: -C * B + s * s - 3 * s + t,
        (2, 2, 0): lambda: (C * C * ((s * s + t * t) // 2 - 2 * t) + C * (-2 * s * s * t + s * s - 3 * t * t + 12 * t)
                            + s * s * (s * s + 4 * t - 12)),
        (2, 2, 1): lambda: s * (C * (2 - t) + s * s + 4 * t - 12),
    }
    return table[(a, b, odd)]()


def d2(a, b, A, B, C):
    r = 1
    for k in range(a):
        r *= A - k * (k + 1)
    for k in range(b):
        r *= B - k * (k + 1)
    for k in range(a + b):
        r *= C - k * (k + 1)
    return r


def _sgn(v):
    return (v > 0) - (v < 0)


def closed_form_sq_sign(a, b, x, y, z):
    """(sign, square) of F_ab(x, y, z) from the closed form (exact)."""
    if x < a or y < b or z < a + b or z < abs(x - y) or z > x + y:
        return 0, Fraction(0)
    L = x + y + z
    A, B, C = x * (x + 1), y * (y + 1), z * (z + 1)
    N = numerator(a, b, L & 1, A, B, C)
    if L % 2 == 0:
        st, t2 = threej_sq_sign(x, y, z, 0, 0, 0)
    else:
        _, y2 = threej_sq_sign(x, y, z + 1, 0, 0, 0)
        t2 = y2 * (L + 2) * (L + 1 - 2 * x) * (L + 1 - 2 * y) * (L - 2 * z)
        st = -1 if ((L + 1) // 2) % 2 else 1
    return st * _sgn(N), t2 * N * N / (4 * d2(a, b, A, B, C))


def canonical(m1, m2):
    """(rotation, flip, a, b): (l1 l2 l3; m1 m2 m3) = [(-1)^L if flip] F_ab(rotated l)."""
    ms = (m1, m2, -m1 - m2)
    for r in range(3):
        p, q = ms[r], ms[(r + 1) % 3]
        if p >= 0 and q >= 0 and p <= 2 and q <= 2:
            return r, 0, p, q
        if p <= 0 and q <= 0 and -p <= 2 and -q <= 2:
            return r, 1, -p, -q
    return None


AB = [(a, b) for a in range(3) for b in range(3)]


@pytest.mark.parametrize("a,b", AB)
def test_closed_forms_exact_small(a, b):
    """Every (x, y, z) with x, y <= 13: squares equal, signs equal."""
    n = 0
    for x in range(0, 14):
        for y in range(0, 14):
            for z in range(abs(x - y), x + y + 1):
                sr, qr = threej_sq_sign(x, y, z, a, b, -a - b)
                sc, qc = closed_form_sq_sign(a, b, x, y, z)
                assert qr == qc, (a, b, x, y, z)
                assert sr == sc, (a, b, x, y, z)
                n += qr != 0
    assert n > 200


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (1, 2), (2, 1)])
def test_closed_forms_exact_larger(a, b):
    """x, y in 38..41 and in the corner z << x = y (where a floating-point
    chain of the lowering relation loses digits)."""
    cases = [(x, y, z) for x in range(38, 42) for y in range(38, 42) for z in range(abs(x - y), x + y + 1, 3)]
    cases += [(60, 60, z) for z in range(0, 12)] + [(61, 60, z) for z in range(1, 12)]
    for (x, y, z) in cases:
        sr, qr = threej_sq_sign(x, y, z, a, b, -a - b)
        sc, qc = closed_form_sq_sign(a, b, x, y, z)
        assert qr == qc and sr == sc, (a, b, x, y, z)


def _g(p):
    return Fraction(comb(2 * p, p), 4 ** p)


def test_w_table_form():
    """W^2 = 8 p1 p2 p3 (L+2) g(p1) g(p2) g(p3) h(P'), h(P) = 1/((2P+1) g(P)),
    P' = (L+1)/2 and p_i = P' - l_i, equals the (x, y, z+1; 0 0 0) form for
    odd L (each of the three neighbouring (0 0 0) symbols gives it)."""
    n = 0
    for x in range(0, 16):
        for y in range(0, 16):
            for z in range(abs(x - y) + 1, x + y, 2):
                L = x + y + z
                P = (L + 1) // 2
                p = [P - x, P - y, P - z]
                w2 = 8 * p[0] * p[1] * p[2] * (L + 2) * _g(p[0]) * _g(p[1]) * _g(p[2]) / ((2 * P + 1) * _g(P))
                for (u, v, w, k) in ((x, y, z + 1, z), (x + 1, y, z, x), (x, y + 1, z, y)):
                    _, y2 = threej_sq_sign(u, v, w, 0, 0, 0)
                    others = [l for l in (x, y, z)]
                    others.remove(k)
                    assert w2 == y2 * (L + 2) * (L - 2 * k) * (L + 1 - 2 * others[0]) * (L + 1 - 2 * others[1])
                n += 1
    assert n > 300


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (2, 1), (1, 2)])
def test_lowering_relation(a, b):
    """The relation that carries the App. B lines into the quadrant, with
    exact symbols (50-digit products of exact square roots)."""
    import mpmath
    mpmath.mp.dps = 50

    def f(p, q, x, y, z):
        sg, sq = threej_sq_sign(x, y, z, p, q, -p - q)
        return sg * mpmath.sqrt(mpmath.mpf(sq.numerator) / sq.denominator)

    for x in range(0, 11):
        for y in range(0, 11):
            for z in range(abs(x - y), x + y + 1):
                lhs = (mpmath.sqrt(max((x + a) * (x - a + 1), 0)) * f(a - 1, b, x, y, z)
                       + mpmath.sqrt(max((y + b) * (y - b + 1), 0)) * f(a, b - 1, x, y, z)
                       + mpmath.sqrt(max((z + a + b) * (z - a - b + 1), 0)) * f(a, b, x, y, z))
                assert abs(lhs) < mpmath.mpf(10) ** -40, (a, b, x, y, z)


MS = [(1, 1), (-1, -1), (2, 2), (-2, -2), (1, 2), (2, 1), (-2, -1), (2, -1), (-1, 2), (-1, -1), (3, -1),
      (1, -3), (4, -2), (-2, 4), (-4, 2), (0, 2), (0, -2), (2, 0), (-1, 1), (2, -2), (0, 0), (1, 0)]


@pytest.mark.parametrize("m1,m2", MS)
def test_canonical_rotation_and_flip(m1, m2):
    """Rotating the columns and flipping the signs reproduces every symbol."""
    c = canonical(m1, m2)
    assert c is not None
    r, flip, a, b = c
    for l1 in range(0, 9):
        for l2 in range(0, 9):
            for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                ls = (l1, l2, l3)
                x, y, z = ls[r], ls[(r + 1) % 3], ls[(r + 2) % 3]
                sr, qr = threej_sq_sign(l1, l2, l3, m1, m2, -m1 - m2)
                sc, qc = closed_form_sq_sign(a, b, x, y, z)
                if flip and (l1 + l2 + l3) % 2:
                    sc = -sc
                assert qr == qc and sr == sc, (m1, m2, l1, l2, l3)


def test_canonical_rejects_large_pairs():
    for (m1, m2) in [(3, 0), (3, -3), (0, 3), (3, 3), (-3, -1), (5, -1), (3, 1)]:
        assert canonical(m1, m2) is None, (m1, m2)


# --- the oracle's general rows ------------------------------------------------------------

ORACLE_MS = [(1, 1), (2, 2), (1, 2), (2, 1), (-1, -1), (-2, -2), (0, 2), (2, -1), (3, -1), (1, -3), (0, 0),
             (1, -1), (4, -2), (3, 3)]


@pytest.mark.parametrize("m1,m2", ORACLE_MS)
def test_oracle_general_rows_small(oracle_bulk, m1, m2):
    for l1 in range(0, 13):
        for l2 in range(0, 13):
            row = oracle_bulk.threej_row_m(l1, l2, m1, m2)
            jm = abs(l1 - l2)
            assert len(row) == l1 + l2 - jm + 1
            ref = np.array([threej(l1, l2, jm + i, m1, m2, -m1 - m2) for i in range(len(row))])
            assert np.max(np.abs(row - ref)) <= 4e-16 * max(1.0, np.max(np.abs(ref))), (m1, m2, l1, l2)


@pytest.mark.parametrize("l1,l2", [(300, 257), (200, 200), (401, 5), (4, 390), (350, 349)])
def test_oracle_general_rows_sampled(oracle_bulk, l1, l2):
    for (m1, m2) in [(1, 1), (2, 2), (-2, -2), (2, 1)]:
        row = oracle_bulk.threej_row_m(l1, l2, m1, m2)
        n, jm = len(row), abs(l1 - l2)
        big = np.max(np.abs(row))
        for i in sorted({0, 1, 2, 3, 4, 5, n // 3, n // 2, n // 2 + 1, n - 3, n - 2, n - 1}):
            ref = threej(l1, l2, jm + i, m1, m2, -m1 - m2)
            assert abs(row[i] - ref) <= 1e-15 * big, (l1, l2, m1, m2, i)

"""Exact tier of the oracle (TEST INFRASTRUCTURE ONLY): the Wigner 3j symbol
from its definition, and the coupling matrices built from it by brute force.

The 3j symbol is evaluated from the Racah sum (the explicit formula of
Edmonds 1957, eq. 3.7.3, which the paper calls E57) in Python integers, so the
square of every symbol is an exact rational and its sign is exact.  Nothing
here uses recurrences, tables of g(p) or the closed forms of Sec. 3: the point
of this tier is to be the definition itself.

The coupling sums follow Sec. 2 (eqs. K_TT, K_EE) and App. A (Xi_TT, Xi_TE,
Xi_EE, Xi_EB; BB has the EE form): for each (l1, l2) the l3 sum is taken over
the whole triangle |l1-l2| <= l3 <= l1+l2 with the parity projectors
[(1 +- (-1)^L)/2] applied literally.  Sums are exact rationals (the signed
products X*Z of the TE kernel are carried as rationals to 2^-240 absolute
accuracy); the final factor (2 l2 + 1)/(4 pi) is applied in 50-digit
arithmetic and rounded once to float64.
"""
from fractions import Fraction
from functools import lru_cache
from math import isqrt

import mpmath

_SQRT_BITS = 240


@lru_cache(maxsize=None)
def _fact(n: int) -> int:
    if n < 0:
        raise ValueError("factorial of a negative number")
    r = 1
    for i in range(2, n + 1):
        r *= i
    return r


def threej_sq_sign(j1, j2, j3, m1, m2, m3):
    """Return (sign, square) of (j1 j2 j3; m1 m2 m3) for integer arguments.

    ``square`` is an exact ``Fraction``; ``sign`` is -1, 0 or +1.  Symbols that
    violate the selection rules (m sum, triangle, |m| <= j) are exactly zero.
    Racah sum (E57 eq. 3.7.3):

        (-1)^(j1-j2-m3) sqrt(Delta) sqrt(prod (j_i +- m_i)!)
            * sum_t (-1)^t / [t! (j3-j2+t+m1)! (j3-j1+t-m2)!
                              (j1+j2-j3-t)! (j1-t-m1)! (j2-t+m2)!]

    with Delta = (j1+j2-j3)! (j1-j2+j3)! (-j1+j2+j3)! / (j1+j2+j3+1)!.
    """
    if m1 + m2 + m3 != 0:
        return 0, Fraction(0)
    if j1 < 0 or j2 < 0 or j3 < 0:
        return 0, Fraction(0)
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0, Fraction(0)
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0, Fraction(0)
    delta = Fraction(_fact(j1 + j2 - j3) * _fact(j1 - j2 + j3) * _fact(-j1 + j2 + j3),
                     _fact(j1 + j2 + j3 + 1))
    pref = (_fact(j1 + m1) * _fact(j1 - m1) * _fact(j2 + m2) * _fact(j2 - m2)
            * _fact(j3 + m3) * _fact(j3 - m3))
    t_lo = max(0, j2 - j3 - m1, j1 - j3 + m2)
    t_hi = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for t in range(t_lo, t_hi + 1):
        den = (_fact(t) * _fact(j3 - j2 + t + m1) * _fact(j3 - j1 + t - m2)
               * _fact(j1 + j2 - j3 - t) * _fact(j1 - t - m1) * _fact(j2 - t + m2))
        s += Fraction(-1 if t % 2 else 1, den)
    if s == 0:
        return 0, Fraction(0)
    phase = -1 if (j1 - j2 - m3) % 2 else 1
    sign = phase * (1 if s > 0 else -1)
    return sign, delta * pref * s * s


def _sqrt_fraction(q: Fraction) -> Fraction:
    """sqrt of a non-negative rational to 2^-_SQRT_BITS relative accuracy."""
    if q == 0:
        return Fraction(0)
    p, r = q.numerator, q.denominator
    scale = 1 << (2 * _SQRT_BITS)
    return Fraction(isqrt(p * r * scale), r << _SQRT_BITS)


def threej(j1, j2, j3, m1, m2, m3) -> float:
    """The 3j symbol as a float64 (exact value, rounded once)."""
    sg, sq = threej_sq_sign(j1, j2, j3, m1, m2, m3)
    if sg == 0:
        return 0.0
    return float(sg * _sqrt_fraction(sq))


def threej_product(j1, j2, j3, mA, mB):
    """(j1 j2 j3; mA) * (j1 j2 j3; mB) as a Fraction (2^-240 accurate).

    ``mA`` and ``mB`` are (m1, m2, m3) tuples.  The sign is exact.
    """
    sa, qa = threej_sq_sign(j1, j2, j3, *mA)
    sb, qb = threej_sq_sign(j1, j2, j3, *mB)
    if sa == 0 or sb == 0:
        return Fraction(0)
    if mA == mB:
        return qa
    return sa * sb * _sqrt_fraction(qa * qb)


SPECTRA = ("TT", "TE", "EE", "BB", "EB")
M000 = (0, 0, 0)
M220 = (-2, 2, 0)


def coupling_term(spec: str, l1: int, l2: int, l3: int) -> Fraction:
    """S^X(l1, l2, l3) of Sec. 2 / App. A, as a Fraction."""
    L = l1 + l2 + l3
    even = 1 if L % 2 == 0 else 0
    odd = 1 - even
    if spec == "TT":
        return threej_product(l1, l2, l3, M000, M000)
    if spec == "TE":
        return even * threej_product(l1, l2, l3, M000, M220)
    if spec in ("EE", "BB"):
        return even * even * threej_product(l1, l2, l3, M220, M220)
    if spec == "EB":
        return odd * odd * threej_product(l1, l2, l3, M220, M220)
    raise ValueError(spec)


def coupling_exact(lmax: int, W, spec: str, abs_sum: bool = False):
    """Exact K^spec for 0 <= l1, l2 <= lmax as a list of lists of float64.

    ``W`` is the window spectrum the spectrum uses (W_TT for TT, W_TP for TE,
    W_PP for EE/BB/EB), indexed by l3 and of length >= 2*lmax+1.  With
    ``abs_sum`` the absolute values of the terms are summed instead (the
    scale the error metric divides by).
    """
    if len(W) < 2 * lmax + 1:
        raise ValueError("W needs entries up to l = 2*lmax")
    Wq = [Fraction(float(w)) for w in W]
    with mpmath.workdps(50):
        four_pi = 4 * mpmath.pi
        out = []
        for l1 in range(lmax + 1):
            row = []
            for l2 in range(lmax + 1):
                acc = Fraction(0)
                for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                    t = (2 * l3 + 1) * Wq[l3] * coupling_term(spec, l1, l2, l3)
                    acc += abs(t) if abs_sum else t
                val = mpmath.mpf(acc.numerator) / acc.denominator * (2 * l2 + 1) / four_pi
                row.append(float(val))
            out.append(row)
    return out

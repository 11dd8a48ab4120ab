"""Pins for the bulk tier of the oracle (oracle/coupling_oracle.c).

The long-double Schulten--Gordon rows and the K sums built from them are
checked against what mathematics fixes, never against themselves:

* the exact Racah values (oracle/racah.py, itself pinned to sympy) for every
  row with l1, l2 <= 30, and sympy's routine at sampled large l;
* the textbook (0 0 0) closed form (E57 eq. 3.7.17) evaluated with 40-digit
  log-gamma at l up to 6000;
* the single-term Racah values at both ends of each row at l up to 6000;
* orthogonality sums the normalisation does not impose: the even-L half of
  sum (2l3+1)(-2 2 0)^2 is exactly 1/2, and sum (2l3+1)(0 0 0)(-2 2 0) = 0;
* brute-force K at small lmax, the full-sky identity, the flat-W closed
  forms, a single-multipole window, linearity in W and the symmetry of Xi.
"""
import math

import mpmath
import numpy as np
import pytest
from sympy.physics.wigner import wigner_3j

from oracle import racah

SPECS = ("TT", "TE", "EE", "BB", "EB")
W_FOR = {"TT": 0, "TE": 1, "EE": 2, "BB": 2, "EB": 2}


def test_rows_equal_racah_small(oracle_bulk):
    worst = 0.0
    for l1 in range(0, 31):
        for l2 in range(0, 31, 1 if l1 < 8 else 3):
            for m in (0, -1, -2):
                row = oracle_bulk.threej_row(l1, l2, m)
                jmin = abs(l1 - l2)
                exact = np.array([racah.threej(l1, l2, jmin + i, m, -m, 0) for i in range(len(row))])
                worst = max(worst, float(np.max(np.abs(row - exact))))
    assert worst < 1e-16


@pytest.mark.parametrize("l1,l2,l3,m", [(300, 400, 100, -2), (300, 400, 402, -2), (300, 400, 700, 0),
                                        (2, 500, 498, -2), (2, 500, 502, -2), (250, 250, 0, -2),
                                        (250, 250, 1, -2), (250, 250, 250, -2), (37, 600, 601, -2),
                                        (300, 400, 101, -1), (300, 400, 650, -1), (1, 500, 500, -1),
                                        (250, 250, 0, -1), (250, 250, 499, -1)])
def test_rows_equal_sympy_large(oracle_bulk, l1, l2, l3, m):
    row = oracle_bulk.threej_row(l1, l2, m)
    ref = float(wigner_3j(l1, l2, l3, m, -m, 0))
    got = row[l3 - abs(l1 - l2)]
    assert got == pytest.approx(ref, rel=2e-15, abs=1e-300)


def _log_closed_form_000(j1, j2, j3):
    """log|(j1 j2 j3; 0 0 0)| and its sign from E57 eq. 3.7.17 (even J)."""
    g = (j1 + j2 + j3) // 2
    lg = mpmath.loggamma
    v = 0.5 * (lg(2 * g - 2 * j1 + 1) + lg(2 * g - 2 * j2 + 1) + lg(2 * g - 2 * j3 + 1) - lg(2 * g + 2)) \
        + lg(g + 1) - lg(g - j1 + 1) - lg(g - j2 + 1) - lg(g - j3 + 1)
    return v, (-1 if g % 2 else 1)


@pytest.mark.parametrize("l1,l2", [(6000, 6000), (5999, 6000), (100, 6000), (3001, 4444), (2, 5000)])
def test_rows_000_equal_closed_form_large(oracle_bulk, l1, l2):
    row = oracle_bulk.threej_row(l1, l2, 0)
    jmin = abs(l1 - l2)
    picks = np.unique(np.linspace(jmin, l1 + l2, 41).astype(int))
    with mpmath.workdps(40):
        for l3 in picks:
            if (l1 + l2 + l3) % 2:
                assert row[l3 - jmin] == 0.0
                continue
            lv, sg = _log_closed_form_000(l1, l2, int(l3))
            ref = sg * float(mpmath.exp(lv))
            assert row[l3 - jmin] == pytest.approx(ref, rel=3e-15)


@pytest.mark.parametrize("l1,l2", [(6000, 6000), (5999, 6000), (2, 6000), (3001, 4444), (1234, 17)])
@pytest.mark.parametrize("m", [0, -1, -2])
def test_row_ends_equal_single_term_racah(oracle_bulk, l1, l2, m):
    # at l3 = |l1-l2| and l3 = l1+l2 the Racah sum has one term: exact even at l ~ 6000
    row = oracle_bulk.threej_row(l1, l2, m)
    jmin, jmax = abs(l1 - l2), l1 + l2
    for l3, got in ((jmin, row[0]), (jmax, row[-1])):
        sg, sq = racah.threej_sq_sign(l1, l2, l3, m, -m, 0)
        with mpmath.workdps(30):
            ref = sg * float(mpmath.sqrt(mpmath.mpf(sq.numerator) / sq.denominator))
        assert got == pytest.approx(ref, rel=2e-15)


@pytest.mark.parametrize("l1,l2", [(2, 2), (2, 3), (7, 300), (1500, 1500), (6000, 5998), (4000, 6000)])
def test_row_orthogonality_pins(oracle_bulk, l1, l2):
    x = oracle_bulk.threej_row(l1, l2, 0)
    z = oracle_bulk.threej_row(l1, l2, -2)
    l3 = np.arange(abs(l1 - l2), l1 + l2 + 1)
    w = 2.0 * l3 + 1.0
    even = (l1 + l2 + l3) % 2 == 0
    assert math.fsum(w * x * x) == pytest.approx(1.0, abs=1e-14)
    assert math.fsum(w * z * z) == pytest.approx(1.0, abs=1e-14)
    assert math.fsum((w * z * z)[even]) == pytest.approx(0.5, abs=1e-14)   # not imposed by the normalisation
    assert abs(math.fsum(w * x * z)) < 1e-14                                # links the two rows


def _rand_w(n, seed, signed=False):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(n) if signed else rng.uniform(0.05, 2.0, n)
    return w


@pytest.mark.parametrize("signed", [False, True])
def test_coupling_equals_brute_force_exact(oracle_bulk, signed):
    lmax = 9
    Ws = [_rand_w(2 * lmax + 1, 11 + i, signed) for i in range(3)]
    K, A = oracle_bulk.coupling_rows(lmax, *Ws, spectra=SPECS)
    for s_i, s in enumerate(SPECS):
        ref = np.array(racah.coupling_exact(lmax, Ws[W_FOR[s]], s))
        refA = np.array(racah.coupling_exact(lmax, Ws[W_FOR[s]], s, abs_sum=True))
        scale = np.maximum(refA, 1e-300)
        assert np.max(np.abs(K[s_i] - ref) / scale) < 4e-16, s
        assert np.max(np.abs(A[s_i] - refA) / scale) < 4e-16, s
        assert np.all((ref == 0) == (K[s_i] == 0)), s


def test_full_sky_identity(oracle_bulk):
    lmax = 300
    W = np.zeros(2 * lmax + 1)
    W[0] = 4.0 * math.pi
    K, _ = oracle_bulk.coupling_rows(lmax, W, W, W, spectra=SPECS)
    eye = np.eye(lmax + 1)
    pol_eye = eye.copy()
    pol_eye[:2, :2] = 0.0
    assert np.max(np.abs(K[0] - eye)) < 2e-15
    for i in (1, 2, 3):
        assert np.max(np.abs(K[i] - pol_eye)) < 2e-15
    assert np.max(np.abs(K[4])) == 0.0


def test_flat_window_closed_forms(oracle_bulk):
    lmax, w = 200, 0.37
    W = np.full(2 * lmax + 1, w)
    K, A = oracle_bulk.coupling_rows(lmax, W, W, W, spectra=SPECS)
    col = (2.0 * np.arange(lmax + 1) + 1.0)[None, :]
    tt = np.broadcast_to(col * w / (4 * math.pi), K[0].shape)
    half = np.broadcast_to(col * w / (8 * math.pi), K[0].shape).copy()
    half[:2, :] = 0.0
    half[:, :2] = 0.0
    assert np.max(np.abs(K[0] - tt) / tt) < 1e-14
    for i in (2, 3, 4):                         # EE, BB and EB each take half of sum (2l3+1)Z^2 = 1
        m = half > 0
        assert np.max(np.abs(K[i][m] - half[m]) / half[m]) < 1e-14
        assert np.all(K[i][~m] == 0.0)
    assert np.max(np.abs(K[1]) / np.maximum(A[1], 1e-300)) < 1e-14   # TE cancels exactly


def test_single_multipole_window(oracle_bulk):
    lmax, L0 = 150, 37
    W = np.zeros(2 * lmax + 1)
    W[L0] = 1.0
    K, _ = oracle_bulk.coupling_rows(lmax, W, W, W, rows=[20, 90, 150], spectra=("TT", "TE", "EE"))
    for ri, l1 in enumerate((20, 90, 150)):
        for l2 in (l1 - 30, l1 - 1, l1 + 0, l1 + 2, l1 + 37):
            if l2 < 0 or l2 > lmax:
                continue
            x = float(wigner_3j(l1, l2, L0, 0, 0, 0))
            z = float(wigner_3j(l1, l2, L0, -2, 2, 0))
            even = (l1 + l2 + L0) % 2 == 0
            pref = (2 * l2 + 1) * (2 * L0 + 1) / (4 * math.pi)
            for si, ref in enumerate((pref * x * x, pref * x * z * even, pref * z * z * even)):
                assert K[si, ri, l2] == pytest.approx(ref, rel=1e-14, abs=1e-300)


def test_linearity_symmetry_and_band(oracle_bulk):
    lmax = 120
    W1, W2 = _rand_w(2 * lmax + 1, 3), _rand_w(2 * lmax + 1, 4)
    a, b = 0.75, 2.5
    K1, A1 = oracle_bulk.coupling_rows(lmax, W1, W1, W1, spectra=SPECS)
    K2, A2 = oracle_bulk.coupling_rows(lmax, W2, W2, W2, spectra=SPECS)
    K12, _ = oracle_bulk.coupling_rows(lmax, a * W1 + b * W2, a * W1 + b * W2, a * W1 + b * W2, spectra=SPECS)
    scale = a * A1 + b * A2 + 1e-300
    assert np.max(np.abs(K12 - (a * K1 + b * K2)) / scale) < 1e-14
    col = 2.0 * np.arange(lmax + 1) + 1.0
    for i in range(len(SPECS)):
        xi = K1[i] / col[None, :]
        assert np.max(np.abs(xi - xi.T) / (A1[i] / col[None, :] + 1e-300)) < 1e-14
    assert np.array_equal(K1[2], K1[3])                       # BB has the EE form
    # band restriction = zeroing W outside the band
    lo, hi = 10, 60
    Wb = W1.copy()
    Wb[:lo] = 0.0
    Wb[hi + 1:] = 0.0
    Kb, Ab = oracle_bulk.coupling_rows(lmax, W1, W1, W1, spectra=SPECS, l3_range=(lo, hi))
    Kz, _ = oracle_bulk.coupling_rows(lmax, Wb, Wb, Wb, spectra=SPECS)
    assert np.max(np.abs(Kb - Kz) / (Ab + 1e-300)) < 1e-15
    l1, l2 = np.meshgrid(np.arange(lmax + 1), np.arange(lmax + 1), indexing="ij")
    assert np.all(Kb[:, np.abs(l1 - l2) > hi] == 0.0)


# ---- band-limited tier: forward recursion from the exact lower end ---------

@pytest.mark.parametrize("l1,l2", [(3, 7), (10, 10), (2, 2), (50, 80), (300, 305), (999, 1999), (2, 600),
                                   (4000, 4400), (6000, 5000)])
@pytest.mark.parametrize("m", [0, -2])
def test_forward_rows_equal_two_sided(oracle_bulk, l1, l2, m):
    full = oracle_bulk.threej_row(l1, l2, m)
    hi = min(l1 + l2, abs(l1 - l2) + 1200)
    fw = oracle_bulk.threej_row_forward(l1, l2, m, hi)
    ref = full[:len(fw)]
    assert np.max(np.abs(fw - ref)) <= 2e-14 * np.max(np.abs(full))


@pytest.mark.parametrize("l1,l2,l3,m", [(5000, 5600, 600, -2), (5000, 5600, 602, 0), (5000, 5600, 640, -2),
                                        (9000, 8500, 500, -2), (9000, 8500, 520, 0)])
def test_forward_rows_equal_sympy_large(oracle_bulk, l1, l2, l3, m):
    fw = oracle_bulk.threej_row_forward(l1, l2, m, l3)
    ref = float(wigner_3j(l1, l2, l3, m, -m, 0))
    assert fw[-1] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("lmax,lo,hi", [(400, 0, 100), (400, 17, 90), (300, 0, 600)])
def test_band_rows_equal_restricted_full_rows(oracle_bulk, lmax, lo, hi):
    Ws = [_rand_w(2 * lmax + 1, 50 + i) for i in range(3)]
    rows = [0, 1, 2, 3, 57, 150, 299, lmax - 1, lmax]
    Kf, Af = oracle_bulk.coupling_rows(lmax, *Ws, rows=rows, spectra=SPECS, l3_range=(lo, hi))
    Kb, Ab = oracle_bulk.coupling_rows(lmax, *Ws, rows=rows, spectra=SPECS, l3_range=(lo, hi), band_forward=True)
    assert np.max(np.abs(Kb - Kf) / (Af + 1e-300)) < 1e-13
    assert np.array_equal(Kf == 0.0, Kb == 0.0)


@pytest.mark.parametrize("l1,l2", [(1, 1), (1, 2), (7, 300), (1500, 1500), (6000, 5998), (4000, 6000)])
def test_row_orthogonality_pins_spin1(oracle_bulk, l1, l2):
    """(-1 1 0) rows: the even-L half of sum (2l3+1)(-1 1 0)^2 is 1/2 (the even
    projector is [(-1 1 0) + (1 -1 0)]/2), and the row is orthogonal to the
    (0 0 0) and (-2 2 0) rows (different m)."""
    x = oracle_bulk.threej_row(l1, l2, 0)
    y = oracle_bulk.threej_row(l1, l2, -1)
    z = oracle_bulk.threej_row(l1, l2, -2)
    l3 = np.arange(abs(l1 - l2), l1 + l2 + 1)
    w = 2.0 * l3 + 1.0
    even = (l1 + l2 + l3) % 2 == 0
    assert math.fsum(w * y * y) == pytest.approx(1.0, abs=1e-14)
    assert math.fsum((w * y * y)[even]) == pytest.approx(0.5, abs=1e-14)
    assert abs(math.fsum(w * x * y)) < 1e-14
    assert abs(math.fsum(w * y * z)) < 1e-14

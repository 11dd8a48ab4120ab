"""Pins of the oracle's binned MASTER solve (oracle/master.py), on the CPU.

* Round trips: the pseudo-spectra are made from known spectra by the
  relations of Sec. 2 eq. pseudo_cl written as separate matrix products
  (C~^EE = K^EE C^EE + K^EB C^BB, C~^BB = K^EB C^EE + K^BB C^BB), so a
  transposed operand or a misplaced block in the solver fails.
* Full sky: K^TT = identity, so binned K = identity and the solution is C~_b.
* Flat window: K^TT_{l1 l2} = (2 l2 + 1) w / (4 pi) (the closed form pinned for
  the coupling oracle), whose binned form is w (hi'^2 - lo'^2) / (4 pi) for the
  column bin [lo', hi').
* Binning of a spectrum: constants stay constant, a linear C_l gives the bin
  midpoint value.
"""
import math

import numpy as np

from oracle import master


def _well_conditioned(n, rng):
    return np.eye(n) + 0.3 * rng.standard_normal((n, n)) / math.sqrt(n)


def test_round_trip_tt():
    rng = np.random.default_rng(0)
    K = _well_conditioned(37, rng)
    C = rng.standard_normal(37)
    assert np.allclose(master.solve_tt(K, K @ C), C, rtol=0, atol=1e-12)
    Cs = rng.standard_normal((4, 37))
    got = master.solve_tt(K, (K @ Cs.T).T)
    assert np.allclose(got, Cs, rtol=0, atol=1e-12)


def test_round_trip_pol_blocks():
    rng = np.random.default_rng(1)
    n = 23
    Kee, Kbb = _well_conditioned(n, rng), _well_conditioned(n, rng)
    Keb = 0.05 * rng.standard_normal((n, n))          # E/B leakage, small
    Cee, Cbb = rng.standard_normal(n), rng.standard_normal(n)
    ct_ee = Kee @ Cee + Keb @ Cbb
    ct_bb = Keb @ Cee + Kbb @ Cbb
    ee, bb = master.solve_pol(Kee, Kbb, Keb, ct_ee, ct_bb)
    assert np.allclose(ee, Cee, rtol=0, atol=1e-12)
    assert np.allclose(bb, Cbb, rtol=0, atol=1e-12)
    # a non-symmetric leakage block catches a transposed placement
    assert not np.allclose(Keb, Keb.T)


def test_full_sky_identity():
    lmax = 40
    edges = [0, 2, 7, 20, 33, 41]
    Kb = master.bin_matrix(np.eye(lmax + 1), edges)
    assert np.array_equal(Kb, np.eye(len(edges) - 1))
    ct = np.arange(lmax + 1, dtype=float) ** 1.5
    ctb = master.bin_spectrum(ct, edges)
    assert np.allclose(master.solve_tt(Kb, ctb), ctb, rtol=1e-15, atol=0)


def test_flat_window_binned_closed_form():
    lmax, w = 60, 0.37
    l = np.arange(lmax + 1)
    K = np.broadcast_to((2 * l + 1) * w / (4 * math.pi), (lmax + 1, lmax + 1))
    edges = [0, 5, 6, 30, 61]
    Kb = master.bin_matrix(K, edges)
    for b in range(4):
        for c in range(4):
            lo, hi = edges[c], edges[c + 1]
            assert math.isclose(Kb[b, c], w * (hi * hi - lo * lo) / (4 * math.pi), rel_tol=1e-14)


def test_bin_spectrum_constant_and_linear():
    edges = [0, 3, 4, 10, 25]
    assert np.allclose(master.bin_spectrum(np.full(25, 2.5), edges), 2.5, rtol=0, atol=0)
    l = np.arange(25, dtype=float)
    mid = [(edges[b] + edges[b + 1] - 1) / 2 for b in range(4)]
    assert np.allclose(master.bin_spectrum(l, edges), mid, rtol=1e-15, atol=0)
    two = master.bin_spectrum(np.stack([l, 2 * l]), edges)
    assert two.shape == (2, 4) and np.allclose(two[1], 2 * two[0])

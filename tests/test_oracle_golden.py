"""Regression against the stored fixtures of tests/golden (written by
tests/golden/make_golden.py from the exact oracle tier), and a check that the
pins catch plausible mistakes planted in a copy of the exact oracle."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import racah

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_threej_fixture():
    n = 0
    with open(os.path.join(GOLD, "threej_small_exact.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            l1, l2, l3, m, sg, sq = line.split()
            got = racah.threej_sq_sign(int(l1), int(l2), int(l3), int(m), -int(m), 0)
            assert got == (int(sg), Fraction(sq)), line
            n += 1
    assert n == 978


def test_coupling_fixture_against_bulk(oracle_bulk):
    lmax = 6
    W = np.array([1.0 / (l + 1) for l in range(2 * lmax + 1)])
    ref = {}
    with open(os.path.join(GOLD, "coupling_small_exact.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            s, l1, l2, v = line.split()
            ref.setdefault(s, np.zeros((lmax + 1, lmax + 1)))[int(l1), int(l2)] = float(v)
    specs = racah.SPECTRA
    K, A = oracle_bulk.coupling_rows(lmax, W, W, W, spectra=specs)
    for i, s in enumerate(specs):
        assert np.max(np.abs(K[i] - ref[s]) / np.maximum(A[i], 1e-300)) < 4e-16, s


# ---- planted mistakes (in a copy of the exact oracle, on the CPU) ----------

def _K(lmax, W, term):
    out = np.zeros((lmax + 1, lmax + 1))
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            acc = 0.0
            for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                acc += term(l1, l2, l3) * W[l3]
            out[l1, l2] = acc
    return out


def _good(spec):
    def term(l1, l2, l3):
        return (2 * l2 + 1) * (2 * l3 + 1) * float(racah.coupling_term(spec, l1, l2, l3)) / (4 * math.pi)
    return term


MUTANTS = {
    "dropped (2 l3 + 1)": lambda l1, l2, l3: (2 * l2 + 1) * float(racah.coupling_term("TT", l1, l2, l3)) / (4 * math.pi),
    "(2 l1 + 1) for (2 l2 + 1)": lambda l1, l2, l3: (2 * l1 + 1) * (2 * l3 + 1) * float(racah.coupling_term("TT", l1, l2, l3)) / (4 * math.pi),
    "TE sign flipped": lambda l1, l2, l3: -(2 * l2 + 1) * (2 * l3 + 1) * float(racah.coupling_term("TE", l1, l2, l3)) / (4 * math.pi),
    "EE without the parity projector": lambda l1, l2, l3: (2 * l2 + 1) * (2 * l3 + 1) * float(racah.threej_product(l1, l2, l3, racah.M220, racah.M220)) / (4 * math.pi),
    "(0 0 0) with m3 = 1": lambda l1, l2, l3: (2 * l2 + 1) * (2 * l3 + 1) * float(racah.threej_product(l1, l2, l3, (0, -1, 1), (0, -1, 1))) / (4 * math.pi),
}
MUTANT_SPEC = {"dropped (2 l3 + 1)": "TT", "(2 l1 + 1) for (2 l2 + 1)": "TT", "TE sign flipped": "TE",
               "EE without the parity projector": "EE", "(0 0 0) with m3 = 1": "TT"}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    """Each mutant fails at least one pin that the real oracle passes: the
    full-sky identity, the flat-window closed forms, or an asymmetric-W
    brute-force element (the role the golden values play)."""
    lmax = 5
    spec = MUTANT_SPEC[name]
    fs = np.zeros(2 * lmax + 1)
    fs[0] = 4 * math.pi
    flat = np.full(2 * lmax + 1, 0.3)
    ramp = np.array([1.0 / (l + 1) for l in range(2 * lmax + 1)])

    def pins_hold(term):
        ok = True
        Kfs = _K(lmax, fs, term)
        eye = np.eye(lmax + 1)
        if spec != "TT":
            eye[:2, :2] = 0.0
        ok &= np.allclose(Kfs, eye, atol=1e-13)
        Kf = _K(lmax, flat, term)
        col = (2.0 * np.arange(lmax + 1) + 1.0)[None, :]
        if spec == "TT":
            ok &= np.allclose(Kf, np.broadcast_to(col * 0.3 / (4 * math.pi), Kf.shape), rtol=1e-13)
        elif spec == "EE":
            ref = np.broadcast_to(col * 0.3 / (8 * math.pi), Kf.shape).copy()
            ref[:2, :] = 0
            ref[:, :2] = 0
            ok &= np.allclose(Kf, ref, rtol=1e-13, atol=1e-15)
        Kr = _K(lmax, ramp, term)
        ref = np.array(racah.coupling_exact(lmax, ramp, spec))
        ok &= np.allclose(Kr, ref, rtol=1e-13, atol=1e-15)
        return bool(ok)

    assert pins_hold(_good(spec))
    assert not pins_hold(MUTANTS[name])

"""Helpers for the parity tests: the error metric and the oracle comparison.

err = max over compared elements of |K - K_ref| / A_ref, where
A_ref = (2 l2 + 1)/(4 pi) sum_l3 (2 l3 + 1) |W S| is the sum of the absolute
values of the terms (for TT/EE/BB with W >= 0 this is the plain relative
error; for TE, whose terms change sign, it is the condition-aware one).
Elements whose reference is exactly 0 (A_ref = 0: polarization at l < 2,
outside a band) must be exactly 0.
"""
import numpy as np

TOL_FP64 = 1e-12
TOL_FP32C = 1e-6
# BF16x3 matrix-core form: each operand is split into bfloat16 hi + lo
# (8 significant bits each, round to nearest), so |x - hi - lo| <= 2^-16 |x|;
# the three kept products hi*hi + hi*lo + lo*hi miss lo*lo and the two split
# residues, each at most 2^-16 of the product: 3 * 2^-16 = 4.58e-5 per term,
# which bounds the sum's error relative to A_ref (the sum of |terms|).  On top
# of it the float32 generation and accumulation, budgeted at 1e-6 as for the
# float32 forms.
TOL_BF16X3 = 3 * 2.0 ** -16 + 1e-6


def parity_error(K, K_ref, A_ref):
    """Return (max relative error, number of exact-zero violations)."""
    K = np.asarray(K, dtype=np.float64)
    zero = A_ref == 0
    bad_zero = int(np.count_nonzero(K[zero] != 0.0))
    nz = ~zero
    err = float(np.max(np.abs(K[nz] - K_ref[nz]) / A_ref[nz])) if np.any(nz) else 0.0
    return err, bad_zero


def assert_parity(K, K_ref, A_ref, tol, what=""):
    err, bad = parity_error(K, K_ref, A_ref)
    assert bad == 0, "%s: %d elements should be exactly 0" % (what, bad)
    assert err <= tol, "%s: max relative error %.3e > %.1e" % (what, err, tol)
    return err

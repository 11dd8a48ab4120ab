"""Seeded synthetic window spectra (inputs only; none of the method's arithmetic).

The paper benchmarks on the ACT DR6 survey window, whose power spectrum W_l is
needed for l <= 2*lmax (Sec. 4).  That map is not available here, so every
workload uses a steeply falling, strictly positive synthetic spectrum of the
same shape:

    W_0 = 4 pi f_sky,                                   f_sky = 0.4
    W_l = W_0 (l + 1)^-2 exp(-(l/l_c)^2) exp(0.1 z_l),   l >= 1,

with z = numpy.random.default_rng(seed).standard_normal(2*lmax + 1) (a
log-normal scatter of width 0.1).  Band-limited windows are set to exactly 0
above their cut.  Seeds follow seed = 1000*workload + 10*mask + spectrum with
spectrum 0/1/2 for the TT/TP/PP windows.

This module is shared by the tests, the benchmark and the smoke check; the
oracle and the HIP path both receive its arrays as plain inputs.
"""
import math

import numpy as np

F_SKY = 0.4

# name -> description of each standard workload
WORKLOADS = {
    0: dict(name="tt_lmax256_fp64", lmax=256, spectra=("TT",), lc=(100.0, 100.0, 100.0),
            precision="fp64", n_masks=1),
    1: dict(name="pol4_lmax2000_fp64", lmax=2000, spectra=("TT", "TE", "EE", "BB"),
            lc=(300.0, 250.0, 200.0), precision="fp64", n_masks=1),
    2: dict(name="pol4_lmax6000_fp32c", lmax=6000, spectra=("TT", "TE", "EE", "BB"),
            lc=(1500.0, 1500.0, 1500.0), precision="fp32c", n_masks=1),
    3: dict(name="batched32_lmax500to4000", lmax=None, spectra=("TT", "TE", "EE", "BB"),
            lc=None, precision="mfma", n_masks=32),
    4: dict(name="band_lmax10000_cut1000_bin50", lmax=10000, spectra=("TT", "EE", "BB"),
            lc=(250.0, 250.0, 250.0), precision="fp32c", n_masks=8, l_cut=1000, bin_width=50,
            n_bins=200),
}


def seed_for(workload: int, mask: int, spectrum: int) -> int:
    return 1000 * workload + 10 * mask + spectrum


def window_spectrum(lmax: int, lc: float, seed: int, l_cut=None, f_sky: float = F_SKY) -> np.ndarray:
    """W_l for l = 0 .. 2*lmax (float64), as in the module docstring."""
    n = 2 * lmax + 1
    z = np.random.default_rng(seed).standard_normal(n)
    ell = np.arange(n, dtype=np.float64)
    w0 = 4.0 * math.pi * f_sky
    w = w0 * (ell + 1.0) ** -2 * np.exp(-(ell / lc) ** 2) * np.exp(0.1 * z)
    w[0] = w0
    if l_cut is not None:
        w[int(l_cut) + 1:] = 0.0
    return w


def full_sky(lmax: int) -> np.ndarray:
    """The full-sky window: W_0 = 4 pi, W_l = 0 otherwise (K = identity)."""
    w = np.zeros(2 * lmax + 1)
    w[0] = 4.0 * math.pi
    return w


def workload_windows(workload: int, mask: int = 0, lmax=None):
    """(W_TT, W_TP, W_PP) of a standard workload (float64 numpy arrays)."""
    spec = WORKLOADS[workload]
    if workload == 3:
        lmaxes = batched_lmaxes()
        lm = lmaxes[mask] if lmax is None else lmax
        lcs = (lm / 4.0,) * 3
    else:
        lm = spec["lmax"] if lmax is None else lmax
        lcs = spec["lc"]
    cut = spec.get("l_cut")
    return tuple(window_spectrum(lm, lcs[s], seed_for(workload, mask, s), l_cut=cut) for s in range(3))


def batched_lmaxes(n: int = 32) -> np.ndarray:
    """Uneven lmax of the batched workload: uniform integers in [500, 4000]."""
    return np.random.default_rng(3000).integers(500, 4001, n)


def sample_rows(lmax: int, fraction: float = 0.01, seed=None, minimum: int = 5) -> np.ndarray:
    """Rows checked against the oracle at full size: a seeded draw without
    replacement of max(minimum, fraction*(lmax+1)) rows, plus both ends."""
    rng = np.random.default_rng(lmax if seed is None else seed)
    n = max(minimum, int(round(fraction * (lmax + 1))))
    rows = set(rng.choice(lmax + 1, size=min(n, lmax + 1), replace=False).tolist())
    rows.update({0, 1, 2, lmax})
    return np.array(sorted(r for r in rows if 0 <= r <= lmax), dtype=np.int32)

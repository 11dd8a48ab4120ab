"""Bulk tier of the oracle (TEST INFRASTRUCTURE ONLY): ctypes access to the
long-double Schulten--Gordon implementation in ``coupling_oracle.c``.

``build()`` compiles ``liboracle.so`` next to this file with gcc/OpenMP.
Nothing from the product package is imported or linked here.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coupling_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SPEC_BITS = {"TT": 1, "TE": 2, "EE": 4, "BB": 8, "EB": 16}
SPEC_ORDER = ("TT", "TE", "EE", "BB", "EB")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_threej_row.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_int]
        lib.oracle_threej_row.restype = ctypes.c_int
        lib.oracle_coupling_rows.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_coupling_rows.restype = ctypes.c_int
        lib.oracle_coupling_rows_upper.argtypes = lib.oracle_coupling_rows.argtypes + [ctypes.c_int]
        lib.oracle_coupling_rows_upper.restype = ctypes.c_int
        lib.oracle_band_rows.argtypes = lib.oracle_coupling_rows.argtypes
        lib.oracle_band_rows.restype = ctypes.c_int
        lib.oracle_threej_row_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_void_p, ctypes.c_int]
        lib.oracle_threej_row_forward.restype = ctypes.c_int
        lib.oracle_threej_row_m.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_int]
        lib.oracle_threej_row_m.restype = ctypes.c_int
        _lib = lib
    return _lib


def threej_row(l1: int, l2: int, m: int) -> np.ndarray:
    """(l1 l2 l3; m -m 0) for l3 = |l1-l2| .. l1+l2 (m = 0, -1 or -2)."""
    n = l1 + l2 - abs(l1 - l2) + 1
    out = np.zeros(n, dtype=np.float64)
    rc = _load().oracle_threej_row(int(l1), int(l2), int(m), out.ctypes.data, n)
    if rc != n:
        raise RuntimeError("oracle_threej_row failed (%d)" % rc)
    return out


def threej_row_forward(l1: int, l2: int, m: int, l3_hi: int) -> np.ndarray:
    """(l1 l2 l3; m -m 0) for l3 = |l1-l2| .. min(l1+l2, l3_hi), by the forward
    recursion from the exact single-term value at the lower end."""
    jmin = abs(l1 - l2)
    n = min(l1 + l2, l3_hi) - jmin + 1
    if n <= 0:
        return np.zeros(0)
    out = np.zeros(n, dtype=np.float64)
    rc = _load().oracle_threej_row_forward(int(l1), int(l2), int(m), int(l3_hi), out.ctypes.data, n)
    if rc != n:
        raise RuntimeError("oracle_threej_row_forward failed (%d)" % rc)
    return out


def threej_row_m(l1: int, l2: int, m1: int, m2: int) -> np.ndarray:
    """(l1 l2 l3; m1 m2 -m1-m2) for l3 = |l1-l2| .. l1+l2 (0 where l3 < |m1+m2|)."""
    n = l1 + l2 - abs(l1 - l2) + 1
    out = np.zeros(n, dtype=np.float64)
    rc = _load().oracle_threej_row_m(int(l1), int(l2), int(m1), int(m2), out.ctypes.data, n)
    if rc != n:
        raise RuntimeError("oracle_threej_row_m failed (%d)" % rc)
    return out


def _as_f64(w):
    if w is None:
        return None
    return np.ascontiguousarray(np.asarray(w, dtype=np.float64))


def coupling_rows(lmax, W_TT=None, W_TP=None, W_PP=None, rows=None, spectra=("TT",),
                  l3_range=None, n_threads=0, with_abs=True, band_forward=False, upper=False):
    """K rows (and the |term| sums) for the requested l1 rows and spectra.

    Returns ``(K, A)`` with shapes [len(spectra), len(rows), lmax+1]; spectra
    are returned in the order given.  ``l3_range=(lo, hi)`` restricts the l3
    sum (band-limited kernels).  ``band_forward`` builds each row only up to
    l3 = hi by the forward recursion from its exact lower end (cost O(hi) per
    element instead of O(l1 + l2)); it requires ``l3_range``.  ``upper``
    evaluates only the entries l2 >= l1 of each row and leaves the others 0
    (full-recursion rows only).
    """
    spectra = tuple(spectra)
    bits = 0
    for s in spectra:
        bits |= SPEC_BITS[s]
    order = [s for s in SPEC_ORDER if bits & SPEC_BITS[s]]
    rows = np.ascontiguousarray(np.arange(lmax + 1) if rows is None else rows, dtype=np.int32)
    ws = [_as_f64(W_TT), _as_f64(W_TP), _as_f64(W_PP)]
    w_len = min(len(w) for w in ws if w is not None)
    lo, hi = (0, 1 << 30) if l3_range is None else (int(l3_range[0]), int(l3_range[1]))
    K = np.zeros((len(order), len(rows), lmax + 1), dtype=np.float64)
    A = np.zeros_like(K) if with_abs else None
    ptr = [w.ctypes.data if w is not None else None for w in ws]
    if band_forward and l3_range is None:
        raise ValueError("band_forward needs l3_range")
    if band_forward and upper:
        raise ValueError("upper applies to full-recursion rows only")
    args = [int(lmax), ptr[0], ptr[1], ptr[2], int(w_len), lo, hi, rows.ctypes.data, len(rows), bits,
            K.ctypes.data, A.ctypes.data if A is not None else None, int(n_threads)]
    if band_forward:
        rc = _load().oracle_band_rows(*args)
    elif upper:
        rc = _load().oracle_coupling_rows_upper(*args, 1)
    else:
        rc = _load().oracle_coupling_rows(*args)
    if rc != 0:
        raise RuntimeError("oracle_coupling_rows failed (%d)" % rc)
    idx = [order.index(s) for s in spectra]
    return K[idx], (A[idx] if A is not None else None)

"""Python binding of libcouple (include/couple.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of ``libcouple.so``;
this module converts torch-ROCm tensors and streams to the C ABI's pointers
and raises ``CoupleError`` with the library's message on failure.  If the
library has not been built, importing the functions works but every call
raises (there is no fallback path).

Function names follow the C ABI: ``couple_init``, ``couple_free``,
``couple_last_error``, ``couple_matrix``, ``couple_band``,
``couple_band_batched``, ``couple_matrix_batched`` (with ``couple_reserve_batched``,
the tile setters and ``couple_autotune_batched``), ``couple_bin_spectra``,
``couple_master_solve``, ``couple_threej_rows``, ``couple_threej_rows_m``, ``couple_tables`` and the
profiling hooks.  ``xi=True`` sets the COUPLE_XI output flag.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcouple.so")

COUPLE_OK, COUPLE_EINVAL, COUPLE_ENOMEM, COUPLE_EDEVICE, COUPLE_ENOTSUP = 0, -1, -2, -3, -4
TT, TE, EE, BB, EB = 1, 2, 4, 8, 16
XI = 256            # output-form flag: the symmetric kernels Xi_X instead of K^X = (2 l2 + 1) Xi_X
SPECTRUM_BITS = {"TT": TT, "TE": TE, "EE": EE, "BB": BB, "EB": EB}
SPECTRUM_ORDER = ("TT", "TE", "EE", "BB", "EB")
PRECISIONS = {"fp64": 0, "fp32c": 1, "mfma_fp32": 2, "mfma_bf16x3": 3}
LMAX_LIMIT = 16384
NOALLOC_SOLVE_DOUBLES = 1 << 22     # COUPLE_NOALLOC_SOLVE_DOUBLES: the static solve workspace (32 MiB)


class CoupleError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("couple error %d: %s" % (code, message))
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcouple.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CoupleError(COUPLE_EDEVICE, "%s is not built; run python -m paper_2602_15605_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp, i, u, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p
    lib.couple_init.argtypes = [i, ctypes.POINTER(vp)]
    lib.couple_init.restype = i
    lib.couple_free.argtypes = [vp]
    lib.couple_free.restype = None
    lib.couple_last_error.argtypes = [vp]
    lib.couple_last_error.restype = ctypes.c_char_p
    lib.couple_lmax_max.argtypes = [vp]
    lib.couple_lmax_max.restype = i
    lib.couple_matrix.argtypes = [vp, dp, dp, dp, i, i, u, i, dp, vp]
    lib.couple_matrix.restype = i
    lib.couple_band.argtypes = [vp, i, i, dp, dp, dp, i, i, u, i, vp, i, dp, vp]
    lib.couple_band.restype = i
    lib.couple_band_batched.argtypes = [vp, i, i, i, vp, vp, vp, i, i, u, i, vp, i, dp, vp]
    lib.couple_band_batched.restype = i
    lib.couple_reserve_batched.argtypes = [vp, i, vp]
    lib.couple_reserve_batched.restype = i
    lib.couple_matrix_batched.argtypes = [vp, i, vp, vp, vp, vp, vp, u, i, vp, vp]
    lib.couple_matrix_batched.restype = i
    lib.couple_set_batched_tiles.argtypes = [vp, i, i, i]
    lib.couple_set_batched_tiles.restype = i
    lib.couple_get_batched_tiles.argtypes = [vp, i, vp, vp]
    lib.couple_get_batched_tiles.restype = i
    lib.couple_autotune_batched.argtypes = [vp, i, i, vp, vp, vp, vp, vp, u, vp, vp, vp, vp, vp]
    lib.couple_autotune_batched.restype = i
    lib.couple_tables.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.couple_tables.restype = i
    lib.couple_threej_rows.argtypes = [vp, i, i, vp, vp, dp, ctypes.c_longlong, vp]
    lib.couple_threej_rows.restype = i
    lib.couple_threej_rows_m.argtypes = [vp, i, i, i, vp, vp, dp, ctypes.c_longlong, vp]
    lib.couple_threej_rows_m.restype = i
    lib.couple_bin_spectra.argtypes = [vp, i, dp, i, vp, i, dp, vp]
    lib.couple_bin_spectra.restype = i
    lib.couple_master_solve.argtypes = [vp, i, i, dp, i, dp, dp, dp, vp]
    lib.couple_master_solve.restype = i
    lib.couple_master_solve_noalloc.argtypes = [vp, i, i, dp, i, dp, dp, vp]
    lib.couple_master_solve_noalloc.restype = i
    lib.couple_profile.argtypes = [vp, i]
    lib.couple_profile.restype = i
    lib.couple_profile_read.argtypes = [vp, vp, vp]
    lib.couple_profile_read.restype = i
    _lib = lib
    return lib


class Context:
    """An initialised couple_ctx (tables + workspace on the current device)."""

    def __init__(self, handle: int, lmax_max: int):
        self.handle = handle
        self.lmax_max = lmax_max

    def __del__(self):
        try:
            couple_free(self)
        except Exception:
            pass


def couple_last_error(ctx=None) -> str:
    lib = load_library()
    msg = lib.couple_last_error(ctx.handle if ctx is not None else None)
    return msg.decode() if msg else ""


def _check(rc, ctx):
    if rc != COUPLE_OK:
        raise CoupleError(rc, couple_last_error(ctx))


def couple_init(lmax_max: int) -> Context:
    lib = load_library()
    h = ctypes.c_void_p()
    rc = lib.couple_init(int(lmax_max), ctypes.byref(h))
    if rc != COUPLE_OK:
        raise CoupleError(rc, couple_last_error(None))
    return Context(h.value, int(lmax_max))


def couple_free(ctx: Context) -> None:
    if ctx is not None and ctx.handle:
        load_library().couple_free(ctx.handle)
        ctx.handle = None


def _spectra_bits(spectra, xi=False) -> int:
    if isinstance(spectra, int):
        bits = spectra
    else:
        bits = 0
        for s in spectra:
            bits |= SPECTRUM_BITS[s]
    return bits | (XI if xi else 0)


def _n_spec(bits: int) -> int:
    return bin(bits & 0x1F).count("1")


def _dev_ptr(t, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise CoupleError(COUPLE_EINVAL, "%s must be a contiguous float64 tensor on the GPU" % name)
    return t.data_ptr()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def couple_matrix(ctx, W_TT, W_TP, W_PP, lmax, spectra=("TT", "TE", "EE", "BB"), precision="fp64",
                  out=None, stream=None, xi=False):
    """K matrices [n_spec, lmax+1, lmax+1] (float64 tensor on the GPU).

    ``W_*`` are float64 GPU tensors of length >= 2*lmax+1 (None where unused).
    ``xi=True`` returns the symmetric kernels Xi_X (COUPLE_XI) instead of K^X.
    Asynchronous on ``stream`` (default: torch's current stream).
    """
    import torch
    bits = _spectra_bits(spectra, xi)
    ns = _n_spec(bits)
    if out is None:
        dev = next(w.device for w in (W_TT, W_TP, W_PP) if w is not None)
        out = torch.empty((max(ns, 1), lmax + 1, lmax + 1), dtype=torch.float64, device=dev)
    elif out.numel() < ns * (lmax + 1) ** 2:
        raise CoupleError(COUPLE_EINVAL, "out is too small")
    ws = [W_TT, W_TP, W_PP]
    w_len = min(int(w.numel()) for w in ws if w is not None)
    rc = load_library().couple_matrix(ctx.handle, _dev_ptr(W_TT, "W_TT"), _dev_ptr(W_TP, "W_TP"),
                                      _dev_ptr(W_PP, "W_PP"), w_len, int(lmax), bits,
                                      PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision),
                                      _dev_ptr(out, "out"), _stream_handle(stream))
    _check(rc, ctx)
    return out


def couple_band(ctx, l3_lo, l3_hi, W_TT, W_TP, W_PP, lmax, spectra=("TT", "EE", "BB"), precision="fp64",
                bin_edges=None, out=None, stream=None, xi=False):
    """Band-limited K (only l3_lo <= l3 <= l3_hi in the sum), optionally binned.

    ``bin_edges``: host sequence of n_bins+1 increasing multipoles, or None.
    ``xi=True``: the symmetric kernels Xi_X instead of K^X.
    Returns [n_spec, lmax+1, lmax+1] or [n_spec, n_bins, n_bins].
    """
    import torch
    bits = _spectra_bits(spectra, xi)
    ns = _n_spec(bits)
    edges = None
    n_bins = 0
    if bin_edges is not None:
        edges = np.ascontiguousarray(np.asarray(bin_edges, dtype=np.int32))
        n_bins = len(edges) - 1
    shape = (max(ns, 1), n_bins, n_bins) if edges is not None else (max(ns, 1), lmax + 1, lmax + 1)
    if out is None:
        dev = next(w.device for w in (W_TT, W_TP, W_PP) if w is not None)
        out = torch.empty(shape, dtype=torch.float64, device=dev)
    elif out.numel() < int(np.prod(shape)):
        raise CoupleError(COUPLE_EINVAL, "out is too small")
    ws = [W_TT, W_TP, W_PP]
    w_len = min(int(w.numel()) for w in ws if w is not None)
    rc = load_library().couple_band(ctx.handle, int(l3_lo), int(l3_hi), _dev_ptr(W_TT, "W_TT"),
                                    _dev_ptr(W_TP, "W_TP"), _dev_ptr(W_PP, "W_PP"), w_len, int(lmax), bits,
                                    PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision),
                                    edges.ctypes.data if edges is not None else None, n_bins,
                                    _dev_ptr(out, "out"), _stream_handle(stream))
    _check(rc, ctx)
    return out


def _ptr_array(tensors, name):
    if tensors is None:
        return None, None
    arr = (ctypes.c_void_p * len(tensors))(*[_dev_ptr(t, name) for t in tensors])
    return arr, len(tensors)


def couple_band_batched(ctx, l3_lo, l3_hi, W_TT, W_TP, W_PP, lmax, spectra=("TT", "EE", "BB"),
                        precision="fp64", bin_edges=None, out=None, stream=None, xi=False):
    """couple_band for a list of masks: ``W_*`` are lists of GPU tensors (or None).

    Returns [n_masks, n_spec, ...] with the couple_band layout per mask.  The
    masks share strip launches (up to four per launch; EB in an odd-L launch
    of its own); every mask's result is bitwise that of couple_band.
    """
    import torch
    bits = _spectra_bits(spectra, xi)
    ns = _n_spec(bits)
    lists = [W_TT, W_TP, W_PP]
    n_masks = next(len(w) for w in lists if w is not None)
    edges = None
    n_bins = 0
    if bin_edges is not None:
        edges = np.ascontiguousarray(np.asarray(bin_edges, dtype=np.int32))
        n_bins = len(edges) - 1
    shape = (n_masks, max(ns, 1)) + ((n_bins, n_bins) if edges is not None else (lmax + 1, lmax + 1))
    if out is None:
        dev = next(w[0].device for w in lists if w is not None)
        out = torch.empty(shape, dtype=torch.float64, device=dev)
    elif out.numel() < int(np.prod(shape)):
        raise CoupleError(COUPLE_EINVAL, "out is too small")
    arrs = [_ptr_array(w, n)[0] for w, n in zip(lists, ("W_TT", "W_TP", "W_PP"))]
    w_len = min(int(t.numel()) for w in lists if w is not None for t in w)
    rc = load_library().couple_band_batched(
        ctx.handle, n_masks, int(l3_lo), int(l3_hi), *[ctypes.cast(a, ctypes.c_void_p) if a is not None else None
                                                        for a in arrs],
        w_len, int(lmax), bits, PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision),
        edges.ctypes.data if edges is not None else None, n_bins, _dev_ptr(out, "out"), _stream_handle(stream))
    _check(rc, ctx)
    return out


def couple_reserve_batched(ctx, lmax_list) -> None:
    """Size the context's batched workspace for masks of these lmax."""
    lm = np.ascontiguousarray(np.asarray(lmax_list, dtype=np.int32))
    _check(load_library().couple_reserve_batched(ctx.handle, len(lm), lm.ctypes.data), ctx)


def couple_matrix_batched(ctx, lmax_list, W_TT, W_TP, W_PP, spectra=("TT", "TE", "EE", "BB"),
                          precision="mfma_fp32", outs=None, stream=None, xi=False):
    """Coupling matrices for a list of masks of uneven lmax in one call.

    ``W_*`` are lists of float64 GPU tensors (or None); returns a list of
    [n_spec, lmax_m+1, lmax_m+1] tensors (Xi_X with ``xi=True``).
    ``precision``: "mfma_fp32" / "mfma_bf16x3" contract on the matrix cores
    (couple_reserve_batched first); "fp32c" / "fp64" run the multi-mask strip
    (masks sorted by lmax share launches), each mask bitwise equal to
    couple_matrix.
    """
    import torch
    bits = _spectra_bits(spectra, xi)
    ns = max(_n_spec(bits), 1)
    lm = np.ascontiguousarray(np.asarray(lmax_list, dtype=np.int32))
    n = len(lm)
    lists = [W_TT, W_TP, W_PP]
    dev = next(w[0].device for w in lists if w is not None)
    if outs is None:
        outs = [torch.empty((ns, int(L) + 1, int(L) + 1), dtype=torch.float64, device=dev) for L in lm]
    elif len(outs) != n or any(o.numel() < ns * (int(L) + 1) ** 2 for o, L in zip(outs, lm)):
        raise CoupleError(COUPLE_EINVAL, "outs must hold one [n_spec, lmax+1, lmax+1] tensor per mask")
    wl = np.ascontiguousarray(np.array([min(int(w[m].numel()) for w in lists if w is not None) for m in range(n)],
                                       dtype=np.int32))
    arrs = [_ptr_array(w, nm)[0] for w, nm in zip(lists, ("W_TT", "W_TP", "W_PP"))]
    optr = (ctypes.c_void_p * n)(*[_dev_ptr(o, "out") for o in outs])
    prec = PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)
    rc = load_library().couple_matrix_batched(
        ctx.handle, n, lm.ctypes.data, *[ctypes.cast(a, ctypes.c_void_p) if a is not None else None for a in arrs],
        wl.ctypes.data, bits, prec, ctypes.cast(optr, ctypes.c_void_p), _stream_handle(stream))
    _check(rc, ctx)
    return outs


def _prec(precision):
    return PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)


def couple_set_batched_tiles(ctx, row_tiles: int, flush: int, precision="mfma_fp32") -> None:
    _check(load_library().couple_set_batched_tiles(ctx.handle, _prec(precision), int(row_tiles), int(flush)), ctx)


def couple_get_batched_tiles(ctx, precision="mfma_fp32"):
    tm, fl = ctypes.c_int(), ctypes.c_int()
    _check(load_library().couple_get_batched_tiles(ctx.handle, _prec(precision), ctypes.byref(tm),
                                                   ctypes.byref(fl)), ctx)
    return tm.value, fl.value


def couple_autotune_batched(ctx, lmax_list, W_TT, W_TP, W_PP, spectra=("TT", "TE", "EE", "BB"), outs=None,
                            stream=None, precision="mfma_fp32"):
    """Time the batched kernel's tile shapes on this batch; keep and return the best
    as (row_tiles, flush, ms)."""
    import torch
    bits = _spectra_bits(spectra)
    ns = max(_n_spec(bits), 1)
    lm = np.ascontiguousarray(np.asarray(lmax_list, dtype=np.int32))
    n = len(lm)
    lists = [W_TT, W_TP, W_PP]
    dev = next(w[0].device for w in lists if w is not None)
    if outs is None:
        outs = [torch.empty((ns, int(L) + 1, int(L) + 1), dtype=torch.float64, device=dev) for L in lm]
    elif len(outs) != n or any(o.numel() < ns * (int(L) + 1) ** 2 for o, L in zip(outs, lm)):
        raise CoupleError(COUPLE_EINVAL, "outs must hold one [n_spec, lmax+1, lmax+1] tensor per mask")
    wl = np.ascontiguousarray(np.array([min(int(w[m].numel()) for w in lists if w is not None) for m in range(n)],
                                       dtype=np.int32))
    arrs = [_ptr_array(w, nm)[0] for w, nm in zip(lists, ("W_TT", "W_TP", "W_PP"))]
    optr = (ctypes.c_void_p * n)(*[_dev_ptr(o, "out") for o in outs])
    tm, fl, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    rc = load_library().couple_autotune_batched(
        ctx.handle, _prec(precision), n, lm.ctypes.data, *[ctypes.cast(a, ctypes.c_void_p) if a is not None else None for a in arrs],
        wl.ctypes.data, bits, ctypes.cast(optr, ctypes.c_void_p), _stream_handle(stream), ctypes.byref(tm),
        ctypes.byref(fl), ctypes.byref(ms))
    _check(rc, ctx)
    return tm.value, fl.value, ms.value


def couple_threej_rows(ctx, l1, l2, m, stride=None, out=None, stream=None):
    """Rows of (l1 l2 l3; -m m 0), m = 0, 1, 2, for l3 = |l1-l2| .. l1+l2.

    ``l1``, ``l2``: sequences or int32 GPU tensors of equal length.  Returns a
    float64 GPU tensor [n_pairs, stride]; row p holds the symbols from
    l3 = |l1[p]-l2[p]| on, 0 past the row's end.  ``stride`` defaults to the
    longest row, 2 max(min(l1, l2)) + 1.
    """
    t1, t2, n, stride, out = _rows_args(l1, l2, stride, out)
    rc = load_library().couple_threej_rows(ctx.handle, int(m), n, t1.data_ptr(), t2.data_ptr(), _dev_ptr(out, "out"),
                                           int(stride), _stream_handle(stream))
    _check(rc, ctx)
    return out


def couple_threej_rows_m(ctx, l1, l2, m1, m2, stride=None, out=None, stream=None):
    """Rows of (l1 l2 l3; m1 m2 -m1-m2) for l3 = |l1-l2| .. l1+l2, for the
    small-m families (e.g. (1 1 -2), (2 2 -4), their m-flips and permutations).

    Arguments, layout and return value as ``couple_threej_rows``.
    """
    t1, t2, n, stride, out = _rows_args(l1, l2, stride, out)
    rc = load_library().couple_threej_rows_m(ctx.handle, int(m1), int(m2), n, t1.data_ptr(), t2.data_ptr(),
                                             _dev_ptr(out, "out"), int(stride), _stream_handle(stream))
    _check(rc, ctx)
    return out


def _rows_args(l1, l2, stride, out):
    import torch
    dev = torch.device("cuda")
    t1 = l1 if isinstance(l1, torch.Tensor) else torch.as_tensor(np.asarray(l1, dtype=np.int32))
    t2 = l2 if isinstance(l2, torch.Tensor) else torch.as_tensor(np.asarray(l2, dtype=np.int32))
    t1 = t1.to(device=dev, dtype=torch.int32).contiguous()
    t2 = t2.to(device=dev, dtype=torch.int32).contiguous()
    if t1.numel() != t2.numel():
        raise CoupleError(COUPLE_EINVAL, "l1 and l2 differ in length")
    n = int(t1.numel())
    if stride is None:
        stride = 2 * int(torch.minimum(t1, t2).max().item()) + 1 if n else 1
    if out is None:
        out = torch.empty((n, int(stride)), dtype=torch.float64, device=dev)
    elif out.numel() < n * int(stride):
        raise CoupleError(COUPLE_EINVAL, "out holds %d entries, needs %d" % (out.numel(), n * int(stride)))
    return t1, t2, n, int(stride), out


def couple_bin_spectra(ctx, cl, bin_edges, out=None, stream=None):
    """Binned pseudo-spectra C~_b = (1/n_b) sum_{l in b} C~_l (couple_band's row-bin rule).

    ``cl``: float64 GPU tensor [n_spec, cl_len] (or [cl_len]); ``bin_edges`` a host
    sequence of n_bins+1 increasing multipoles.  Returns [n_spec, n_bins] (or [n_bins]).
    """
    import torch
    one = cl.dim() == 1
    c2 = cl.reshape(1, -1) if one else cl
    if not c2.is_contiguous():
        raise CoupleError(COUPLE_EINVAL, "cl must be contiguous")
    edges = np.ascontiguousarray(np.asarray(bin_edges, dtype=np.int32))
    n_bins = len(edges) - 1
    if out is None:
        out = torch.empty((c2.shape[0], n_bins), dtype=torch.float64, device=cl.device)
    elif out.numel() < c2.shape[0] * n_bins:
        raise CoupleError(COUPLE_EINVAL, "out holds %d entries, needs %d" % (out.numel(), c2.shape[0] * n_bins))
    rc = load_library().couple_bin_spectra(ctx.handle, int(c2.shape[0]), _dev_ptr(c2, "cl"), int(c2.shape[1]),
                                           edges.ctypes.data, n_bins, _dev_ptr(out, "out"), _stream_handle(stream))
    _check(rc, ctx)
    return out.reshape(-1) if one else out


def couple_master_solve(ctx, K, rhs, pol=False, work=None, out=None, stream=None):
    """Solve the binned MASTER system K_{b b'} C_{b'} = C~_b.

    ``pol=False``: ``K`` is [n, n] (or [1, n, n]); ``rhs`` [n] or [n_rhs, n].
    ``pol=True``: ``K`` is [3, n, n] = binned (EE, BB, EB) as couple_band writes them
    for spectra ("EE", "BB", "EB"); ``rhs`` [2n] or [n_rhs, 2n] (EE then BB).
    Returns the solution with the shape of ``rhs``.
    """
    import torch
    n = int(K.shape[-1])
    m = 2 * n if pol else n
    one = rhs.dim() == 1
    r2 = rhs.reshape(1, -1) if one else rhs
    if r2.shape[1] != m:
        raise CoupleError(COUPLE_EINVAL, "rhs has %d entries per system, expected %d" % (r2.shape[1], m))
    if not (K.is_contiguous() and r2.is_contiguous()):
        raise CoupleError(COUPLE_EINVAL, "K and rhs must be contiguous")
    n_rhs = int(r2.shape[0])
    if K.numel() < (3 if pol else 1) * n * n:
        raise CoupleError(COUPLE_EINVAL, "K holds %d entries, expected %d" % (K.numel(), (3 if pol else 1) * n * n))
    if work is None:
        work = torch.empty(m * (m + n_rhs), dtype=torch.float64, device=K.device)
    elif work.numel() < m * (m + n_rhs):
        raise CoupleError(COUPLE_EINVAL, "work holds %d entries, needs %d" % (work.numel(), m * (m + n_rhs)))
    if out is None:
        out = torch.empty((n_rhs, m), dtype=torch.float64, device=K.device)
    elif out.numel() < n_rhs * m:
        raise CoupleError(COUPLE_EINVAL, "out holds %d entries, needs %d" % (out.numel(), n_rhs * m))
    rc = load_library().couple_master_solve(ctx.handle, 1 if pol else 0, n, _dev_ptr(K, "K"), n_rhs,
                                            _dev_ptr(r2, "rhs"), _dev_ptr(work, "work"), _dev_ptr(out, "x"),
                                            _stream_handle(stream))
    _check(rc, ctx)
    return out.reshape(-1) if one else out


def couple_master_solve_noalloc(ctx, K, rhs, pol=False, out=None, stream=None):
    """couple_master_solve with the library's static device workspace instead of
    ``work`` (no allocation in the C call; pass ``out`` to allocate nothing here
    either).  Shapes as couple_master_solve; m * (m + n_rhs) <= NOALLOC_SOLVE_DOUBLES.
    """
    import torch
    n = int(K.shape[-1])
    m = 2 * n if pol else n
    one = rhs.dim() == 1
    r2 = rhs.reshape(1, -1) if one else rhs
    if r2.shape[1] != m:
        raise CoupleError(COUPLE_EINVAL, "rhs has %d entries per system, expected %d" % (r2.shape[1], m))
    if not (K.is_contiguous() and r2.is_contiguous()):
        raise CoupleError(COUPLE_EINVAL, "K and rhs must be contiguous")
    n_rhs = int(r2.shape[0])
    if K.numel() < (3 if pol else 1) * n * n:
        raise CoupleError(COUPLE_EINVAL, "K holds %d entries, expected %d" % (K.numel(), (3 if pol else 1) * n * n))
    if out is None:
        out = torch.empty((n_rhs, m), dtype=torch.float64, device=K.device)
    elif out.numel() < n_rhs * m:
        raise CoupleError(COUPLE_EINVAL, "out holds %d entries, needs %d" % (out.numel(), n_rhs * m))
    rc = load_library().couple_master_solve_noalloc(ctx.handle, 1 if pol else 0, n, _dev_ptr(K, "K"), n_rhs,
                                                    _dev_ptr(r2, "rhs"), _dev_ptr(out, "x"),
                                                    _stream_handle(stream))
    _check(rc, ctx)
    return out.reshape(-1) if one else out


def couple_tables(ctx):
    """Host copies of the look-up tables: dict g, h, cl (float64), gf, hf (float32)."""
    L = ctx.lmax_max
    t = dict(g=np.zeros(L + 1), h=np.zeros(2 * L + 1), cl=np.zeros(L + 1),
             gf=np.zeros(L + 1, dtype=np.float32), hf=np.zeros(2 * L + 1, dtype=np.float32))
    rc = load_library().couple_tables(ctx.handle, t["g"].ctypes.data, t["h"].ctypes.data, t["cl"].ctypes.data,
                                      t["gf"].ctypes.data, t["hf"].ctypes.data)
    _check(rc, ctx)
    return t


N_STAGES = 3
STAGES = ("scale_windows", "strip", "fill")


def couple_profile(ctx, enable: bool) -> None:
    """Measurement hook: record HIP events around every kernel of later calls."""
    _check(load_library().couple_profile(ctx.handle, 1 if enable else 0), ctx)


def couple_profile_read(ctx):
    """{stage: (total_ms, launches)} accumulated since couple_profile(ctx, True)."""
    ms = np.zeros(N_STAGES, dtype=np.float64)
    cnt = np.zeros(N_STAGES, dtype=np.int32)
    _check(load_library().couple_profile_read(ctx.handle, ms.ctypes.data, cnt.ctypes.data), ctx)
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(N_STAGES)}

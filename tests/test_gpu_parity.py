"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 path: every compared element within 1e-12 relative (error metric of
tests/_parity.py).  Full matrices where the oracle finishes in seconds
(several 64-wide tiles and ragged tails), seeded sampled rows at the full
workload sizes, and the invariants that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

from _parity import TOL_FP32C, TOL_FP64, assert_parity, parity_error

pytestmark = pytest.mark.gpu

SPEC4 = ("TT", "TE", "EE", "BB")
W_INDEX = {"TT": 0, "TE": 1, "EE": 2, "BB": 2}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_gpu):
    from paper_2602_15605_amd import couple
    c = couple.couple_init(6000)
    yield c
    couple.couple_free(c)


def _gpu(torch, arr):
    return torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64)).cuda()


def _run(torch, ctx, Ws, lmax, spectra=SPEC4, precision="fp64"):
    from paper_2602_15605_amd import couple
    dW = [_gpu(torch, w) for w in Ws]
    out = couple.couple_matrix(ctx, dW[0], dW[1], dW[2], lmax, spectra=spectra, precision=precision)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    del out
    return res


def _oracle(oracle_bulk, Ws, lmax, spectra=SPEC4, rows=None, l3_range=None):
    return oracle_bulk.coupling_rows(lmax, Ws[0], Ws[1], Ws[2], rows=rows, spectra=spectra, l3_range=l3_range)


def _windows(lmax, seed, kind="positive"):
    rng = np.random.default_rng(seed)
    n = 2 * lmax + 1
    if kind == "positive":
        return [rng.uniform(0.01, 2.0, n) for _ in range(3)]
    return [rng.standard_normal(n) for _ in range(3)]


def test_tables_correctly_rounded(torch_gpu, ctx):
    import mpmath
    from paper_2602_15605_amd import couple
    t = couple.couple_tables(ctx)
    L = ctx.lmax_max
    g_ref = np.zeros(2 * L + 1)
    h_ref = np.zeros(2 * L + 1)
    with mpmath.workdps(60):
        g = mpmath.mpf(1)
        for p in range(2 * L + 1):
            if p:
                g = g * (2 * p - 1) / (2 * p)       # exact definition, 60 digits
            g_ref[p] = float(g)
            h_ref[p] = float(1 / ((2 * p + 1) * g))
    assert np.array_equal(t["g"], g_ref[:L + 1])
    assert np.array_equal(t["h"], h_ref)
    assert np.array_equal(t["gf"], g_ref[:L + 1].astype(np.float32))
    assert np.max(np.abs(t["hf"].astype(np.float64) - h_ref) / h_ref) < 6e-8
    ell = np.arange(L + 1, dtype=np.float64)
    with np.errstate(divide="ignore"):
        cl_ref = np.where(ell >= 2, 1.0 / np.sqrt((ell - 1) * ell * (ell + 1) * (ell + 2)), 0.0)
    assert np.array_equal(t["cl"][:2], [0.0, 0.0])
    assert np.max(np.abs(t["cl"][2:] - cl_ref[2:]) / cl_ref[2:]) < 4e-16


@pytest.mark.parametrize("lmax", [0, 1, 2, 3, 5, 63, 64, 65, 255, 256, 257, 511])
@pytest.mark.parametrize("kind", ["positive", "signed"])
def test_full_matrix_parity_small(torch_gpu, ctx, oracle_bulk, lmax, kind):
    _say("full parity lmax=%d W=%s" % (lmax, kind))
    Ws = _windows(lmax, 100 + lmax, kind)
    K = _run(torch_gpu, ctx, Ws, lmax)
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax)
    for i, s in enumerate(SPEC4):
        assert_parity(K[i], Kr[i], Ar[i], TOL_FP64, "%s lmax=%d" % (s, lmax))
    assert np.array_equal(K[2], K[3])


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
@pytest.mark.parametrize("spectra", [("TT",), ("TE",), ("EE", "BB"), ("TT", "EE"), ("BB",)])
def test_spectra_subsets(torch_gpu, ctx, oracle_bulk, spectra, precision, tol):
    """Each subset runs the kernel mode it selects (TT only; all three even-L
    sums when TE is asked for; TT + EE; EE alone)."""
    lmax = 130
    Ws = _windows(lmax, 7)
    Wuse = [Ws[0] if "TT" in spectra else None, Ws[1] if "TE" in spectra else None,
            Ws[2] if ("EE" in spectra or "BB" in spectra) else None]
    from paper_2602_15605_amd import couple
    dW = [_gpu(torch_gpu, w) if w is not None else None for w in Wuse]
    K = couple.couple_matrix(ctx, dW[0], dW[1], dW[2], lmax, spectra=spectra, precision=precision).cpu().numpy()
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=spectra)
    assert K.shape[0] == len(spectra)
    for i, s in enumerate(spectra):
        assert_parity(K[i], Kr[i], Ar[i], tol, s)


def test_workload0_tt_lmax256(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import synth
    lmax = 256
    Ws = synth.workload_windows(0)
    K = _run(torch_gpu, ctx, Ws, lmax, spectra=("TT",))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=("TT",))
    err = assert_parity(K[0], Kr[0], Ar[0], TOL_FP64, "workload0")
    _say("workload0 TT lmax=256 max rel err %.3e" % err)


def test_full_sky_identity(torch_gpu, ctx):
    from paper_2602_15605_amd import synth
    for lmax in (256, 2000):
        w = synth.full_sky(lmax)
        K = _run(torch_gpu, ctx, [w, w, w], lmax)
        eye = np.eye(lmax + 1)
        pol = eye.copy()
        pol[:2, :2] = 0.0
        assert np.max(np.abs(K[0] - eye)) < 1e-14
        for i in (1, 2, 3):
            assert np.max(np.abs(K[i] - pol)) < 1e-14
            assert np.all(K[i][:2, :] == 0.0) and np.all(K[i][:, :2] == 0.0)


def test_exact_block_small_l(torch_gpu, ctx):
    """Brute force from the Racah sum (exact tier) for l <= 12."""
    from oracle import racah
    lmax = 12
    Ws = _windows(lmax, 5)
    K = _run(torch_gpu, ctx, Ws, lmax)
    for i, s in enumerate(SPEC4):
        ref = np.array(racah.coupling_exact(lmax, Ws[W_INDEX[s]], s))
        refA = np.array(racah.coupling_exact(lmax, Ws[W_INDEX[s]], s, abs_sum=True))
        assert_parity(K[i], ref, refA, TOL_FP64, s)


def test_flat_window_closed_forms(torch_gpu, ctx):
    lmax, w = 1000, 0.21
    W = np.full(2 * lmax + 1, w)
    K = _run(torch_gpu, ctx, [W, W, W], lmax)
    col = (2.0 * np.arange(lmax + 1) + 1.0)[None, :]
    tt = np.broadcast_to(col * w / (4 * math.pi), K[0].shape)
    assert np.max(np.abs(K[0] - tt) / tt) < 1e-12
    half = np.broadcast_to(col * w / (8 * math.pi), K[0].shape)[2:, 2:]
    for i in (2, 3):
        assert np.max(np.abs(K[i][2:, 2:] - half) / half) < 1e-12
    # TE cancels exactly: |K^TE| small against the scale of its terms, which
    # for flat W is bounded by the EE/TT sizes
    assert np.max(np.abs(K[1][2:, 2:]) / tt[2:, 2:]) < 1e-12


def test_workload1_sampled_rows(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import synth
    lmax = 2000
    Ws = synth.workload_windows(1)
    K = _run(torch_gpu, ctx, Ws, lmax)
    rows = synth.sample_rows(lmax)
    _say("workload1: %d rows vs oracle" % len(rows))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, rows=rows)
    for i, s in enumerate(SPEC4):
        err = assert_parity(K[i][rows], Kr[i], Ar[i], TOL_FP64, "workload1 %s" % s)
        _say("workload1 %s max rel err %.3e" % (s, err))
    assert np.array_equal(K[2], K[3])
    # Xi = K / (2 l2 + 1) is symmetric
    col = 2.0 * np.arange(lmax + 1) + 1.0
    for i in range(3):
        xi = K[i] / col[None, :]
        scale = np.abs(xi) + np.abs(xi.T) + 1e-300
        assert np.max(np.abs(xi - xi.T) / scale) < 1e-15


@pytest.mark.parametrize("precision,tol,workload", [("fp64", TOL_FP64, 1), ("fp32c", TOL_FP32C, 2),
                                                     ("fp32c", TOL_FP32C, 1)])
def test_full_matrix_lmax2000(torch_gpu, ctx, oracle_bulk, precision, tol, workload):
    """Every element of the four 2001 x 2001 matrices against the oracle: the
    pol4_lmax2000 windows (l_c = 300, 250, 200) in FP64 and FP32C, and the
    l_c = 1500 windows of the FP32C workload in FP32C.  With l_c = 200 the PP
    window falls below float32's normal range (about 1e-38) from about l3 = 1790 on,
    so the far diagonals of K^EE hold only such terms: FP32C keeps them
    through its per-item power-of-two scales."""
    import os
    import time
    from paper_2602_15605_amd import synth
    lmax = 2000
    Ws = synth.workload_windows(workload, lmax=lmax)
    K = _run(torch_gpu, ctx, Ws, lmax, precision=precision)
    t0 = time.perf_counter()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, spectra=SPEC4, n_threads=min(16, os.cpu_count() or 1))
    _say("full lmax 2000 %s: oracle %.1f s" % (precision, time.perf_counter() - t0))
    for i, s in enumerate(SPEC4):
        err = assert_parity(K[i], Kr[i], Ar[i], tol, "full lmax 2000 %s %s" % (precision, s))
        _say("  %s max rel err %.3e" % (s, err))


@pytest.mark.parametrize("precision,tol,lmax", [("fp32c", TOL_FP32C, 1918), ("fp32c", TOL_FP32C, 1919),
                                                  ("fp64", TOL_FP64, 1321), ("fp64", TOL_FP64, 1322),
                                                  ("fp64", TOL_FP64, 1000), ("fp32c", TOL_FP32C, 1000)])
def test_row_block_switch(torch_gpu, ctx, oracle_bulk, precision, tol, lmax):
    """Both sides of the size below which the strip kernels take 128-row
    blocks (two rows per lane) instead of 256: 1918 / 1919 in FP32C, 1321 /
    1322 in FP64, on sampled rows and both ends, all four spectra and EB.
    The FP32C cases use the l_c = 1500 windows of the FP32C workload."""
    from paper_2602_15605_amd import synth
    spec5 = SPEC4 + ("EB",)
    Ws = synth.workload_windows(1 if precision == "fp64" else 2, lmax=lmax)
    K = _run(torch_gpu, ctx, Ws, lmax, spectra=spec5, precision=precision)
    rows = np.unique(np.concatenate([synth.sample_rows(lmax, fraction=0.02), [lmax - 1, lmax // 3]])).astype(np.int32)
    _say("row block switch %s lmax %d: %d rows" % (precision, lmax, len(rows)))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=spec5, rows=rows)
    for i, s in enumerate(spec5):
        assert_parity(K[i][rows], Kr[i], Ar[i], tol, "%s lmax %d %s" % (precision, lmax, s))


@pytest.mark.parametrize("lmax", [1918, 2100])
def test_fp32c_window_tails_below_float32(torch_gpu, ctx, oracle_bulk, lmax):
    """FP32C with windows whose tails leave float32's range: the pol4_lmax2000
    windows taken to lmax 1918 (128-row blocks) and 2100 (256-row blocks),
    where W'_PP(l3) is below 1e-38 from about l3 = 1790 on and below 1e-60 at the
    far corner.  Sampled rows (rows 0 .. 2 reach the last diagonals), all four
    spectra and EB; the far corner of every spectrum is non-zero."""
    from paper_2602_15605_amd import synth
    spec5 = SPEC4 + ("EB",)
    Ws = synth.workload_windows(1, lmax=lmax)
    assert Ws[2][2 * lmax] < 1e-60
    K = _run(torch_gpu, ctx, Ws, lmax, spectra=spec5, precision="fp32c")
    rows = np.unique(np.concatenate([synth.sample_rows(lmax, fraction=0.02), [lmax - 1, lmax // 3]])).astype(np.int32)
    _say("fp32c window tails lmax %d: %d rows" % (lmax, len(rows)))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=spec5, rows=rows)
    for i, s in enumerate(spec5):
        err = assert_parity(K[i][rows], Kr[i], Ar[i], TOL_FP32C, "fp32c tails lmax %d %s" % (lmax, s))
        _say("  %s max rel err %.3e" % (s, err))
        assert np.all(K[i][2:5, lmax - 2:] != 0.0), s


def test_workload2_fp64_sampled_rows(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import synth
    lmax = 6000
    Ws = synth.workload_windows(2)
    K = _run(torch_gpu, ctx, Ws, lmax)
    rows = synth.sample_rows(lmax, seed=6000)
    _say("workload2 fp64: %d rows vs oracle" % len(rows))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, rows=rows)
    for i, s in enumerate(SPEC4):
        err = assert_parity(K[i][rows], Kr[i], Ar[i], TOL_FP64, "workload2 fp64 %s" % s)
        _say("workload2 fp64 %s max rel err %.3e" % (s, err))


@pytest.mark.parametrize("lmax,lo,hi", [(300, 0, 40), (300, 17, 90), (257, 0, 514), (400, 100, 100),
                                         (129, 5, 3000)])
def test_band_parity(torch_gpu, ctx, oracle_bulk, lmax, lo, hi):
    from paper_2602_15605_amd import couple
    Ws = _windows(lmax, 31)
    dW = [_gpu(torch_gpu, w) for w in Ws]
    K = couple.couple_band(ctx, lo, hi, dW[0], dW[1], dW[2], lmax, spectra=SPEC4).cpu().numpy()
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, l3_range=(lo, hi))
    for i, s in enumerate(SPEC4):
        assert_parity(K[i], Kr[i], Ar[i], TOL_FP64, "band %s" % s)


def test_band_binned(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import couple
    lmax, lo, hi = 399, 0, 60
    Ws = _windows(lmax, 41)
    edges = np.array([0, 2, 10, 50, 51, 100, 160, 250, 400])
    dW = [_gpu(torch_gpu, w) for w in Ws]
    Kb = couple.couple_band(ctx, lo, hi, dW[0], dW[1], dW[2], lmax, spectra=("TT", "EE", "BB"),
                            bin_edges=edges).cpu().numpy()
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=("TT", "EE", "BB"), l3_range=(lo, hi))
    nb = len(edges) - 1
    for i in range(3):
        ref = np.zeros((nb, nb))
        refA = np.zeros((nb, nb))
        for b in range(nb):
            for c in range(nb):
                blk = (slice(edges[b], edges[b + 1]), slice(edges[c], edges[c + 1]))
                ref[b, c] = Kr[i][blk].sum() / (edges[b + 1] - edges[b])
                refA[b, c] = Ar[i][blk].sum() / (edges[b + 1] - edges[b])
        assert_parity(Kb[i], ref, refA, 1e-12, "binned")


def test_error_codes_with_context(torch_gpu, ctx):
    from paper_2602_15605_amd import couple
    lib = couple.load_library()
    w = _gpu(torch_gpu, np.ones(21))
    out = torch_gpu.empty((4, 11, 11), dtype=torch_gpu.float64, device="cuda")
    p, o = w.data_ptr(), out.data_ptr()
    h = ctx.handle
    s = torch_gpu.cuda.current_stream().cuda_stream
    cases = [
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 15, 0, o, s), 0, ""),
        (lambda: lib.couple_matrix(h, p, p, p, 20, 10, 15, 0, o, s), -1, "w_len"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, -1, 15, 0, o, s), -1, "lmax"),
        (lambda: lib.couple_matrix(h, p, p, p, 100000, 6001, 15, 0, o, s), -1, "lmax"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 0, 0, o, s), -1, "spectra"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 32, 0, o, s), -1, "spectra"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 15, 7, o, s), -1, "precision"),
        (lambda: lib.couple_matrix(h, None, p, p, 21, 10, 15, 0, o, s), -1, "W_TT"),
        (lambda: lib.couple_matrix(h, p, None, p, 21, 10, 2, 0, o, s), -1, "W_TP"),
        (lambda: lib.couple_matrix(h, p, p, None, 21, 10, 8, 0, o, s), -1, "W_PP"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 15, 0, None, s), -1, "out"),
        (lambda: lib.couple_matrix(h, p, p, p, 21, 10, 15, 0, o + 4, s), -1, "aligned"),
        (lambda: lib.couple_matrix(h, None, None, p, 21, 10, 4, 0, o, s), 0, ""),
        (lambda: lib.couple_band(h, 5, 2, p, p, p, 21, 10, 1, 0, None, 0, o, s), -1, "band"),
        (lambda: lib.couple_band(h, -1, 2, p, p, p, 21, 10, 1, 0, None, 0, o, s), -1, "band"),
        (lambda: lib.couple_band(h, 0, 30, p, p, p, 15, 10, 1, 0, None, 0, o, s), -1, "w_len"),
    ]
    for call, want, text in cases:
        rc = call()
        assert rc == want, (rc, want, text)
        if text:
            assert text in couple.couple_last_error(ctx), (text, couple.couple_last_error(ctx))
        else:
            assert couple.couple_last_error(ctx) == ""
    bad_edges = np.array([0, 5, 5, 11], dtype=np.int32)
    rc = lib.couple_band(h, 0, 4, p, p, p, 21, 10, 1, 0, bad_edges.ctypes.data, 3, o, s)
    assert rc == -1 and "increasing" in couple.couple_last_error(ctx)
    bad_edges = np.array([0, 5, 12], dtype=np.int32)
    rc = lib.couple_band(h, 0, 4, p, p, p, 21, 10, 1, 0, bad_edges.ctypes.data, 2, o, s)
    assert rc == -1
    torch_gpu.cuda.synchronize()


def test_nondefault_stream(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import couple
    lmax = 200
    Ws = _windows(lmax, 9)
    st = torch_gpu.cuda.Stream()
    with torch_gpu.cuda.stream(st):
        dW = [_gpu(torch_gpu, w) for w in Ws]
        out = couple.couple_matrix(ctx, *dW, lmax, stream=st)
    st.synchronize()
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax)
    for i in range(4):
        assert_parity(out[i].cpu().numpy(), Kr[i], Ar[i], TOL_FP64, "stream")


# ---- FP32-compensated path: <= 1e-6 relative --------------------------------

@pytest.mark.parametrize("lmax", [2, 5, 64, 129, 256, 700])
def test_fp32c_full_matrix_parity(torch_gpu, ctx, oracle_bulk, lmax):
    _say("fp32c full parity lmax=%d" % lmax)
    Ws = _windows(lmax, 300 + lmax)
    K = _run(torch_gpu, ctx, Ws, lmax, precision="fp32c")
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax)
    for i, s in enumerate(SPEC4):
        err = assert_parity(K[i], Kr[i], Ar[i], TOL_FP32C, "fp32c %s lmax=%d" % (s, lmax))
        _say("  %s %.3e" % (s, err))
    assert np.array_equal(K[2], K[3])


def test_fp32c_full_sky_identity(torch_gpu, ctx):
    from paper_2602_15605_amd import synth
    lmax = 1000
    w = synth.full_sky(lmax)
    K = _run(torch_gpu, ctx, [w, w, w], lmax, precision="fp32c")
    eye = np.eye(lmax + 1)
    pol = eye.copy()
    pol[:2, :2] = 0.0
    assert np.max(np.abs(K[0] - eye)) < 1e-6
    for i in (1, 2, 3):
        assert np.max(np.abs(K[i] - pol)) < 1e-6
        assert np.all(K[i][:2, :] == 0.0) and np.all(K[i][:, :2] == 0.0)


def test_workload2_fp32c_sampled_rows(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import synth
    lmax = 6000
    Ws = synth.workload_windows(2)
    K = _run(torch_gpu, ctx, Ws, lmax, precision="fp32c")
    rows = synth.sample_rows(lmax, seed=6000)
    _say("workload2 fp32c: %d rows vs oracle" % len(rows))
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, rows=rows)
    for i, s in enumerate(SPEC4):
        err = assert_parity(K[i][rows], Kr[i], Ar[i], TOL_FP32C, "workload2 fp32c %s" % s)
        _say("workload2 fp32c %s max rel err %.3e" % (s, err))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_graph_replay_matrix_and_band(torch_gpu, ctx, precision):
    """couple_matrix (five spectra) and binned couple_band allocate nothing and
    enqueue kernels only, so a captured graph replays to the eager result, replay
    after replay, with eager work and synchronisations in between."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 300
    Ws = _windows(lmax, 61)
    dW = [_gpu(torch, w) for w in Ws]
    spectra = ("TT", "TE", "EE", "BB", "EB")
    edges = [0, 3, 50, 51, 200, 301]
    eager_k = couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=precision).clone()
    eager_b = couple.couple_band(ctx, 2, 120, *dW, lmax, spectra=spectra, precision=precision,
                                 bin_edges=edges).clone()
    out_k = torch.empty_like(eager_k)
    out_b = torch.empty_like(eager_b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=precision, out=out_k)
        couple.couple_band(ctx, 2, 120, *dW, lmax, spectra=spectra, precision=precision, bin_edges=edges,
                           out=out_b)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=precision, out=out_k)
        couple.couple_band(ctx, 2, 120, *dW, lmax, spectra=spectra, precision=precision, bin_edges=edges,
                           out=out_b)
    for rep in range(4):
        out_k.fill_(float("nan"))
        out_b.fill_(float("nan"))
        x = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_k, eager_k), rep
        assert torch.equal(out_b, eager_b), rep
        del x


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
def test_lmax_limit_sampled_rows(torch_gpu, oracle_bulk, precision, tol):
    """lmax = COUPLE_LMAX_LIMIT (16384), all five spectra, sampled rows including
    l1 = lmax.  l3 reaches 2 lmax = 32768, where the FP32C kernel's exact t split
    needs its rebasing and FP64 evaluates N' beyond 2^53.  Windows with
    l_c = lmax / 2 keep every K element inside the float32 range."""
    from paper_2602_15605_amd import couple, synth
    torch = torch_gpu
    lmax = couple.LMAX_LIMIT
    W = [synth.window_spectrum(lmax, lmax / 2.0, 7000 + s) for s in range(3)]
    spectra = ("TT", "TE", "EE", "BB", "EB")
    rows = np.array([2, 3000, 9001, lmax - 1, lmax])
    c = couple.couple_init(lmax)
    try:
        dW = [_gpu(torch, w) for w in W]
        K = couple.couple_matrix(c, *dW, lmax, spectra=spectra, precision=precision)
        got = K[:, torch.as_tensor(rows).cuda(), :].cpu().numpy()
        del K
    finally:
        couple.couple_free(c)
    torch.cuda.empty_cache()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *W, rows=rows, spectra=spectra)
    for i, s in enumerate(spectra):
        err = assert_parity(got[i], Kr[i], Ar[i], tol, "lmax %d %s %s" % (lmax, precision, s))
        _say("lmax %d %s %s max rel err %.3e" % (lmax, precision, s, err))


@pytest.mark.parametrize("n_bins", [512, 701, 4097])
def test_unit_bins_equal_unbinned(torch_gpu, ctx, n_bins):
    """Bins one multipole wide reproduce the unbinned matrix bitwise, both for
    bin lists carried in the kernel arguments (<= 512 bins) and for longer lists
    staged through the context's pinned buffer.  4097 bins: 4097^2 bin pairs of
    256 work-items exceed 2^32 work-items in one grid dimension, so the bin
    kernel's grid is two-dimensional."""
    from paper_2602_15605_amd import couple
    lmax = n_bins - 1
    Ws = _windows(lmax, 91)
    dW = [_gpu(torch_gpu, w) for w in Ws]
    spectra = ("TT", "TE", "EE", "BB", "EB")
    K = couple.couple_band(ctx, 1, 200, *dW, lmax, spectra=spectra)
    Kb = couple.couple_band(ctx, 1, 200, *dW, lmax, spectra=spectra, bin_edges=np.arange(lmax + 2))
    assert Kb.shape == K.shape
    assert torch_gpu.equal(Kb, K)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_ragged_bins_all_spectra(torch_gpu, ctx, precision):
    """Ragged bins (1 to 301 multipoles wide, so a bin spans several 64-row
    chunks) over all five spectra (four distinct Xi stores), with and without
    a band cut that runs through bins: the binned K is the bin operator
    (row-bin average, column-bin sum) applied to the unbinned K of the same
    call, within 1e-13 of the bin's sum of |K|."""
    from paper_2602_15605_amd import couple
    lmax = 700
    dW = [_gpu(torch_gpu, w) for w in _windows(lmax, 93)]
    spectra = ("TT", "TE", "EE", "BB", "EB")
    edges = [0, 1, 2, 65, 66, 200, 501, 701]
    nb = len(edges) - 1
    for lo, hi in ((0, 2 * lmax), (3, 150)):
        K = couple.couple_band(ctx, lo, hi, *dW, lmax, spectra=spectra, precision=precision).cpu().numpy()
        Kb = couple.couple_band(ctx, lo, hi, *dW, lmax, spectra=spectra, precision=precision,
                                bin_edges=edges).cpu().numpy()
        assert Kb.shape == (5, nb, nb)
        for b in range(nb):
            for c in range(nb):
                blk = K[:, edges[b]:edges[b + 1], edges[c]:edges[c + 1]]
                n = edges[b + 1] - edges[b]
                ref = blk.sum(axis=(1, 2)) / n
                scale = np.abs(blk).sum(axis=(1, 2)) / n
                assert np.all(np.abs(Kb[:, b, c] - ref) <= 1e-13 * scale), (precision, lo, hi, b, c)
                if np.all(blk == 0.0):
                    assert np.all(Kb[:, b, c] == 0.0)
        assert np.array_equal(Kb[2], Kb[3])          # K^BB shares K^EE's sums
        _say("ragged bins %s l3 in [%d, %d]: ok" % (precision, lo, hi))


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
def test_band_tt_only(torch_gpu, ctx, oracle_bulk, precision, tol):
    """K^TT alone, band-limited below lmax (the band grid of the TT-only mode,
    eight rows per lane), against the oracle's band tier."""
    from paper_2602_15605_amd import couple
    lmax, lo, hi = 600, 5, 300
    Ws = _windows(lmax, 61)
    K = couple.couple_band(ctx, lo, hi, _gpu(torch_gpu, Ws[0]), None, None, lmax, spectra=("TT",),
                           precision=precision).cpu().numpy()
    Kr, Ar = _oracle(oracle_bulk, Ws, lmax, spectra=("TT",), l3_range=(lo, hi))
    err = assert_parity(K[0], Kr[0], Ar[0], tol, "band TT %s" % precision)
    _say("band TT only %s max rel err %.3e" % (precision, err))

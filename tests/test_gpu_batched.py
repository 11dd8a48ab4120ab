"""Batched form: many masks of uneven lmax in one call, contracted on the
matrix cores (COUPLE_MFMA_FP32 and COUPLE_MFMA_BF16X3) or through the
multi-mask FP32C strip, checked per mask against the oracle and, for the strip
paths, bitwise against single-mask calls.

The workload is 32 synthetic masks with lmax uniform in [500, 4000]; every
mask is compared on >= 1% of its rows (at least 5, plus rows 0, 1, 2, lmax).
Small full-matrix cases cover the group edges: masks of very different lmax
sharing a 16-mask column group, a second group with one mask, lmax 0..3.
"""
import sys

import numpy as np
import pytest

from _parity import TOL_BF16X3, TOL_FP32C, assert_parity

pytestmark = pytest.mark.gpu

SPEC4 = ("TT", "TE", "EE", "BB")
MFMA = [("mfma_fp32", TOL_FP32C), ("mfma_bf16x3", TOL_BF16X3)]


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
    c = couple.couple_init(4000)
    yield c
    couple.couple_free(c)


def _rand_windows(lmaxes, seed):
    rng = np.random.default_rng(seed)
    return [[rng.uniform(0.05, 1.5, 2 * L + 1) for _ in range(3)] for L in lmaxes]


@pytest.mark.parametrize("precision,tol", MFMA + [("fp32c", TOL_FP32C)])
def test_batched_small_full_parity(torch_gpu, ctx, oracle_bulk, precision, tol):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [257, 3, 64, 0, 65, 200, 1, 130, 17, 2, 255, 100, 31, 32, 33, 150, 90]   # 17 masks: 2 groups
    _say("batched small full parity %s, lmax %s" % (precision, lmaxes))
    Ws = _rand_windows(lmaxes, 5)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=SPEC4, precision=precision)
    torch.cuda.synchronize()
    worst = 0.0
    for m, L in enumerate(lmaxes):
        K = outs[m].cpu().numpy()
        Kr, Ar = oracle_bulk.coupling_rows(L, *Ws[m], spectra=SPEC4)
        for i, s in enumerate(SPEC4):
            worst = max(worst, assert_parity(K[i], Kr[i], Ar[i], tol, "mask %d lmax %d %s" % (m, L, s)))
        assert np.array_equal(K[2], K[3])
    _say("batched small %s: max rel err %.3e" % (precision, worst))


@pytest.mark.parametrize("precision,tol,tm,flush", [("mfma_fp32", TOL_FP32C, 2, 4), ("mfma_fp32", TOL_FP32C, 2, 8),
                                                     ("mfma_fp32", TOL_FP32C, 64, 2), ("mfma_fp32", TOL_FP32C, 128, 2),
                                                     ("mfma_bf16x3", TOL_BF16X3, 2, 4)])
def test_batched_workload3_sampled_rows(torch_gpu, ctx, oracle_bulk, precision, tol, tm, flush):
    """The 32-mask workload in both float32 forms at every flush interval the
    autotuner may pick."""
    from paper_2602_15605_amd import couple, synth
    torch = torch_gpu
    lmaxes = [int(x) for x in synth.batched_lmaxes()]
    _say("workload3 batched %s tiles %d flush %d" % (precision, tm, flush))
    Ws = [synth.workload_windows(3, mask=m) for m in range(len(lmaxes))]
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    saved = couple.couple_get_batched_tiles(ctx, precision=precision)
    couple.couple_set_batched_tiles(ctx, tm, flush, precision=precision)
    try:
        outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=SPEC4, precision=precision)
        torch.cuda.synchronize()
    finally:
        couple.couple_set_batched_tiles(ctx, *saved, precision=precision)
    worst = {s: 0.0 for s in SPEC4}
    for m, L in enumerate(lmaxes):
        rows = synth.sample_rows(L, fraction=0.01, seed=3000 + m, minimum=5)
        got = outs[m][:, torch.as_tensor(rows.astype(np.int64)).cuda(), :].cpu().numpy()
        Kr, Ar = oracle_bulk.coupling_rows(L, *Ws[m], rows=rows, spectra=SPEC4)
        for i, s in enumerate(SPEC4):
            worst[s] = max(worst[s], assert_parity(got[i], Kr[i], Ar[i], tol, "mask %d lmax %d %s" % (m, L, s)))
    _say("workload3 batched %s tiles %d flush %d max rel err: " % (precision, tm, flush)
         + ", ".join("%s %.3e" % kv for kv in worst.items()))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("spectra", [SPEC4, ("TT", "EE", "BB"), ("TT",), ("EE", "BB"), ("TT", "TE"),
                                     ("TT", "TE", "EE", "BB", "EB")])
def test_batched_strip_paths_equal_single_calls(torch_gpu, ctx, precision, spectra):
    """couple_matrix_batched in FP64 and FP32C equals couple_matrix mask by mask,
    bitwise.  It runs the multi-mask strips (FP32C's EB only where every mask's
    one-mask strip runs full lanes, not at these sizes): masks sorted by lmax,
    four per launch (with TE three in FP32C, two in FP64), over the grid of the
    group's largest lmax, so a smaller mask's rows run in other blocks and past
    their own end; their sums still come out bitwise equal (extra all-zero
    blocks leave k - c unchanged through a Kahan step).  With 9 masks of mixed
    lmax (0, 1, equal values)."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [40, 300, 7, 300, 128, 129, 255, 1, 0]
    Ws = _rand_windows(lmaxes, 8)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=spectra, precision=precision)
    for m in range(len(lmaxes)):
        K1 = couple.couple_matrix(ctx, dW[0][m], dW[1][m], dW[2][m], lmaxes[m], spectra=spectra, precision=precision)
        assert torch.equal(outs[m], K1), (m, lmaxes[m])


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_batched_eb_multimask_equal_single_calls(torch_gpu, ctx, precision):
    """Full matrices with EB through the multi-mask odd-L strip, even and odd
    strips per group, equal to couple_matrix bitwise.  FP32C takes masks of lmax
    1792 and up (the one-mask strip's full lanes) in groups whose lmax agree mod 4,
    here {2254, 2250} and {2180, 2100, 1792}, and runs lmax 1791, 300 and 40 one
    by one; FP64 groups all eight."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [2100, 2250, 300, 2180, 2254, 40, 1791, 1792]
    Ws = _rand_windows(lmaxes, 12)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    for spectra in (("TT", "EE", "BB", "EB"), ("EB",)):
        outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=spectra, precision=precision)
        for m in range(len(lmaxes)):
            K1 = couple.couple_matrix(ctx, dW[0][m], dW[1][m], dW[2][m], lmaxes[m], spectra=spectra,
                                      precision=precision)
            assert torch.equal(outs[m], K1), (spectra, m, lmaxes[m])
            del K1
        del outs


def test_batched_fp32c_xi_workspace_waves(torch_gpu, oracle_bulk):
    """FP32C batched masks whose Xi stores exceed the context's Xi workspace and
    no batched workspace: the call runs in waves of groups (here one mask per
    group: two lmax-300 masks need 6 triangles, the workspace holds 4), each
    followed by its fill; results equal single calls bitwise and the oracle."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [300, 300, 299, 150, 300]
    c = couple.couple_init(300)
    try:
        Ws = _rand_windows(lmaxes, 9)
        dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
        outs = couple.couple_matrix_batched(c, lmaxes, dW[0], dW[1], dW[2], spectra=SPEC4, precision="fp32c")
        for m in range(len(lmaxes)):
            K1 = couple.couple_matrix(c, dW[0][m], dW[1][m], dW[2][m], lmaxes[m], spectra=SPEC4, precision="fp32c")
            assert torch.equal(outs[m], K1), m
        K = outs[4].cpu().numpy()
    finally:
        couple.couple_free(c)
    Kr, Ar = oracle_bulk.coupling_rows(300, *Ws[4], spectra=SPEC4)
    for i, s in enumerate(SPEC4):
        assert_parity(K[i], Kr[i], Ar[i], TOL_FP32C, "waves %s" % s)


def test_batched_errors(torch_gpu, ctx):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    w = [torch.ones(81, dtype=torch.float64, device="cuda")]
    with pytest.raises(couple.CoupleError, match="lmax"):
        couple.couple_matrix_batched(ctx, [4001], [torch.ones(8003, dtype=torch.float64, device="cuda")],
                                     None, None, spectra=("TT",))
    with pytest.raises(couple.CoupleError, match="w_len"):
        couple.couple_matrix_batched(ctx, [41], w, None, None, spectra=("TT",))
    with pytest.raises(couple.CoupleError, match="n_masks"):
        couple.couple_reserve_batched(ctx, list(range(65)))
    fresh = couple.couple_init(100)
    try:
        for prec in ("mfma_fp32", "mfma_bf16x3"):
            with pytest.raises(couple.CoupleError, match="couple_reserve_batched"):
                couple.couple_matrix_batched(fresh, [40], w, None, None, spectra=("TT",), precision=prec)
    finally:
        couple.couple_free(fresh)
    with pytest.raises(couple.CoupleError, match="batched tile shape"):
        couple.couple_set_batched_tiles(ctx, 2, 8, precision="fp32c")
    with pytest.raises(couple.CoupleError, match="batched only"):
        couple.couple_matrix(ctx, w[0], None, None, 40, spectra=("TT",), precision="mfma_bf16x3")


F32_SHAPES = [(tm, fl) for tm in (1, 2, 4) for fl in (1, 4, 8, 16)] + [(tm, fl) for tm in (64, 128) for fl in (1, 2, 4)]
BF16_SHAPES = [(tm, fl) for tm in (1, 2, 4) for fl in (1, 2, 4)]


@pytest.mark.parametrize("precision,tol,shapes", [("mfma_fp32", TOL_FP32C, F32_SHAPES),
                                                   ("mfma_bf16x3", TOL_BF16X3, BF16_SHAPES)])
def test_autotune_and_tile_shapes(torch_gpu, ctx, oracle_bulk, precision, tol, shapes):
    """Every tile shape gives a result within the bar; the autotuner keeps one of them."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [300, 77, 1, 190]
    Ws = _rand_windows(lmaxes, 21)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    refs = [oracle_bulk.coupling_rows(L, *Ws[m], spectra=SPEC4) for m, L in enumerate(lmaxes)]
    saved = couple.couple_get_batched_tiles(ctx, precision=precision)
    other = "mfma_bf16x3" if precision == "mfma_fp32" else "mfma_fp32"
    saved_other = couple.couple_get_batched_tiles(ctx, precision=other)
    try:
        for tm, fl in shapes:
            _say("%s row_tiles %d flush %d" % (precision, tm, fl))
            couple.couple_set_batched_tiles(ctx, tm, fl, precision=precision)
            outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], precision=precision)
            for m in range(len(lmaxes)):
                K = outs[m].cpu().numpy()
                for i, s in enumerate(SPEC4):
                    assert_parity(K[i], refs[m][0][i], refs[m][1][i], tol, "tm %d flush %d %s" % (tm, fl, s))
        tm, fl, ms = couple.couple_autotune_batched(ctx, lmaxes, dW[0], dW[1], dW[2], precision=precision)
        assert (tm, fl) in shapes and ms > 0
        assert couple.couple_get_batched_tiles(ctx, precision=precision) == (tm, fl)
        assert couple.couple_get_batched_tiles(ctx, precision=other) == saved_other
        _say("autotune %s picked row_tiles=%d flush=%d (%.3f ms)" % (precision, tm, fl, ms))
        with pytest.raises(couple.CoupleError):
            couple.couple_set_batched_tiles(ctx, 3, 8, precision=precision)
    finally:
        couple.couple_set_batched_tiles(ctx, *saved, precision=precision)


@pytest.mark.parametrize("precision", ["mfma_fp32", "mfma_bf16x3", "fp32c", "fp64"])
def test_batched_graph_replay(torch_gpu, ctx, precision):
    """The batched call is capture-safe: a captured graph replays to the eager result,
    replay after replay, with eager work in between."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [250, 64, 180]
    Ws = _rand_windows(lmaxes, 33)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    eager = [o.clone() for o in couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2],
                                                            precision=precision)]
    outs = [torch.empty_like(o) for o in eager]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], precision=precision, outs=outs)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], precision=precision, outs=outs)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        x = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")  # eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for m in range(len(lmaxes)):
            assert torch.equal(outs[m], eager[m]), (rep, m)
        del x


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_batched_eb_graph_replay(torch_gpu, ctx, precision):
    """With EB the batched FP32C / FP64 call (even and odd-L multi-mask strips,
    lmax 1804 .. 2000, equal mod 4) captures into a graph that replays to the
    eager result, replay after replay, with eager work in between."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [1900, 2000, 1804]
    spectra = ("TT", "EE", "BB", "EB")
    Ws = _rand_windows(lmaxes, 44)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    eager = [o.clone() for o in couple.couple_matrix_batched(ctx, lmaxes, dW[0], None, dW[2], spectra=spectra,
                                                            precision=precision)]
    outs = [torch.empty_like(o) for o in eager]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        couple.couple_matrix_batched(ctx, lmaxes, dW[0], None, dW[2], spectra=spectra, precision=precision,
                                     outs=outs)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        couple.couple_matrix_batched(ctx, lmaxes, dW[0], None, dW[2], spectra=spectra, precision=precision,
                                     outs=outs)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        x = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")  # eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for m in range(len(lmaxes)):
            assert torch.equal(outs[m], eager[m]), (rep, m)
        del x
    K1 = couple.couple_matrix(ctx, dW[0][1], None, dW[2][1], lmaxes[1], spectra=spectra, precision=precision)
    assert torch.equal(outs[1], K1)
    del graph, outs, eager, K1


@pytest.mark.parametrize("precision,tol", MFMA)
def test_batched_64_masks_four_groups(torch_gpu, ctx, oracle_bulk, precision, tol):
    """The largest batch: 64 masks in four column groups (64 fill jobs), with
    repeated, tiny (0, 1) and equal lmax values; every mask's full matrix checked."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    rng = np.random.default_rng(64)
    lmaxes = [int(x) for x in rng.integers(0, 90, 60)] + [0, 1, 89, 89]
    _say("64 masks %s, lmax %d..%d" % (precision, min(lmaxes), max(lmaxes)))
    Ws = _rand_windows(lmaxes, 65)
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=SPEC4, precision=precision)
    torch.cuda.synchronize()
    worst = 0.0
    for m, L in enumerate(lmaxes):
        K = outs[m].cpu().numpy()
        Kr, Ar = oracle_bulk.coupling_rows(L, *Ws[m], spectra=SPEC4)
        for i, s in enumerate(SPEC4):
            worst = max(worst, assert_parity(K[i], Kr[i], Ar[i], tol, "mask %d lmax %d %s" % (m, L, s)))
    _say("64 masks %s: max rel err %.3e" % (precision, worst))

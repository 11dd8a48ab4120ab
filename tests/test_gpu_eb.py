"""The odd-L (EB) coupling matrix on the GPU against the oracle.

S^EB = [(1-(-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2 with W_PP (App. A).  The kernel
uses the odd-J reduction of App. B (eq. 022_rearranged with eq. joneodd and
eq. joneevensimp), an integer row factor times the (0 0 0)^2 of (l1, l2+1,
l3); the oracle evaluates the symbol by recursion.  FP64 within 1e-12 and
FP32C within 1e-6 of the oracle (error metric of tests/_parity.py), plus the
closed forms that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

from _parity import TOL_FP32C, TOL_FP64, assert_parity

pytestmark = pytest.mark.gpu

SPEC5 = ("TT", "TE", "EE", "BB", "EB")


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
    c = couple.couple_init(2000)
    yield c
    couple.couple_free(c)


def _gpu(torch, arr):
    return torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64)).cuda()


def _windows(lmax, seed, kind="positive"):
    rng = np.random.default_rng(seed)
    n = 2 * lmax + 1
    if kind == "positive":
        return [rng.uniform(0.01, 2.0, n) for _ in range(3)]
    return [rng.standard_normal(n) for _ in range(3)]


@pytest.mark.parametrize("lmax", [0, 1, 2, 3, 4, 5, 63, 64, 65, 257, 511])
@pytest.mark.parametrize("kind", ["positive", "signed"])
def test_eb_full_parity_fp64(torch_gpu, ctx, oracle_bulk, lmax, kind):
    from paper_2602_15605_amd import couple
    _say("EB full parity fp64 lmax=%d W=%s" % (lmax, kind))
    Ws = _windows(lmax, 300 + lmax, kind)
    dW = [_gpu(torch_gpu, w) for w in Ws]
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision="fp64").cpu().numpy()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, spectra=SPEC5)
    for i, s in enumerate(SPEC5):
        assert_parity(K[i], Kr[i], Ar[i], TOL_FP64, "%s lmax=%d" % (s, lmax))
    # rows / columns 0 and 1 vanish; the even outputs do not change when EB is added
    assert np.all(K[4][:2, :] == 0.0) and np.all(K[4][:, :2] == 0.0)
    K4 = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5[:4], precision="fp64").cpu().numpy()
    assert np.array_equal(K4, K[:4])


@pytest.mark.parametrize("lmax", [5, 129, 700])
def test_eb_full_parity_fp32c(torch_gpu, ctx, oracle_bulk, lmax):
    from paper_2602_15605_amd import couple
    _say("EB full parity fp32c lmax=%d" % lmax)
    Ws = _windows(lmax, 400 + lmax)
    dW = [_gpu(torch_gpu, w) for w in Ws]
    K = couple.couple_matrix(ctx, None, None, dW[2], lmax, spectra=("EB",), precision="fp32c").cpu().numpy()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, spectra=("EB",))
    err = assert_parity(K[0], Kr[0], Ar[0], TOL_FP32C, "EB fp32c lmax=%d" % lmax)
    _say("  max rel err %.3e" % err)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_eb_only_request(torch_gpu, ctx, oracle_bulk, precision):
    from paper_2602_15605_amd import couple
    lmax = 200
    Ws = _windows(lmax, 17)
    K = couple.couple_matrix(ctx, None, None, _gpu(torch_gpu, Ws[2]), lmax, spectra=("EB",),
                             precision=precision).cpu().numpy()
    assert K.shape == (1, lmax + 1, lmax + 1)
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, spectra=("EB",))
    assert_parity(K[0], Kr[0], Ar[0], TOL_FP64 if precision == "fp64" else TOL_FP32C, "EB only")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_eb_full_sky_and_flat_window(torch_gpu, ctx, precision):
    """Full sky (W_0 = 4 pi, W_l>0 = 0): only l3 = 0 enters, L is even, K^EB = 0
    exactly.  Flat window W_l = w: the odd-L half of sum (2 l3 + 1)(-2 2 0)^2 = 1
    is 1/2, so K^EB = (2 l2 + 1) w / (8 pi) for l1, l2 >= 2."""
    from paper_2602_15605_amd import couple
    lmax = 300
    w = np.zeros(2 * lmax + 1)
    w[0] = 4 * math.pi
    K = couple.couple_matrix(ctx, None, None, _gpu(torch_gpu, w), lmax, spectra=("EB",),
                             precision=precision).cpu().numpy()[0]
    assert np.all(K == 0.0)
    flat = np.full(2 * lmax + 1, 0.7)
    K = couple.couple_matrix(ctx, None, None, _gpu(torch_gpu, flat), lmax, spectra=("EB",),
                             precision=precision).cpu().numpy()[0]
    l2 = np.arange(lmax + 1)
    ref = np.broadcast_to((2 * l2 + 1) * 0.7 / (8 * math.pi), K.shape).copy()
    ref[:2, :] = 0.0
    ref[:, :2] = 0.0
    nz = ref != 0
    tol = TOL_FP64 if precision == "fp64" else TOL_FP32C
    assert np.max(np.abs(K[nz] - ref[nz]) / ref[nz]) < tol
    assert np.all(K[~nz] == 0.0)


@pytest.mark.parametrize("precision,tol,workload", [("fp64", TOL_FP64, 1), ("fp32c", TOL_FP32C, 2)])
def test_eb_workload_sampled_rows(torch_gpu, ctx, oracle_bulk, precision, tol, workload):
    """lmax = 2000, 1% of the rows, all five spectra.  FP64 on the pol4_lmax2000
    windows (l_c = 300/250/200); FP32C on the l_c = 1500 windows of the FP32C
    workload: with l_c = 200, W_l falls to ~1e-50 at l = 2000 and the far
    off-diagonal K elements lie below the float32 range."""
    from paper_2602_15605_amd import couple, synth
    torch = torch_gpu
    lmax = 2000
    W = synth.workload_windows(workload, lmax=lmax)
    dW = [_gpu(torch, w) for w in W]
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision)
    rows = synth.sample_rows(lmax, fraction=0.01, seed=2000, minimum=5)
    got = K[:, torch.as_tensor(rows.astype(np.int64)).cuda(), :].cpu().numpy()
    del K
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *W, rows=rows, spectra=SPEC5)
    for i, s in enumerate(SPEC5):
        err = assert_parity(got[i], Kr[i], Ar[i], tol, "%s %s" % (precision, s))
        _say("workload%d lmax 2000 %s %s max rel err %.3e" % (workload, precision, s, err))


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
def test_eb_band_and_bins(torch_gpu, ctx, oracle_bulk, precision, tol):
    from paper_2602_15605_amd import couple
    lmax, lo, hi = 700, 3, 250
    Ws = _windows(lmax, 29)
    dW = [_gpu(torch_gpu, w) for w in Ws]
    spectra = ("EE", "EB")
    K = couple.couple_band(ctx, lo, hi, None, None, dW[2], lmax, spectra=spectra, precision=precision)
    rows = np.array([0, 1, 2, 3, 100, 249, 250, 251, 400, 699, 700])
    got = K[:, _gpu(torch_gpu, rows).long(), :].cpu().numpy()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, rows=rows, spectra=spectra, l3_range=(lo, hi))
    for i, s in enumerate(spectra):
        assert_parity(got[i], Kr[i], Ar[i], tol, "band %s %s" % (precision, s))
    edges = [0, 2, 30, 100, 101, 400, 701]
    Kb = couple.couple_band(ctx, lo, hi, None, None, dW[2], lmax, spectra=spectra, precision=precision,
                            bin_edges=edges).cpu().numpy()
    Kfull = K.cpu().numpy()
    for b in range(len(edges) - 1):
        for c in range(len(edges) - 1):
            blk = Kfull[:, edges[b]:edges[b + 1], edges[c]:edges[c + 1]]
            ref = blk.sum(axis=(1, 2)) / (edges[b + 1] - edges[b])
            assert np.allclose(Kb[:, b, c], ref, rtol=1e-13, atol=1e-300)


def test_eb_not_in_matrix_core_form(torch_gpu, ctx):
    from paper_2602_15605_amd import couple
    w = [_gpu(torch_gpu, np.ones(201))]
    couple.couple_reserve_batched(ctx, [100])
    for prec in ("mfma_fp32", "mfma_bf16x3"):
        with pytest.raises(couple.CoupleError, match="EB") as e:
            couple.couple_matrix_batched(ctx, [100], None, None, w, spectra=("EB",), precision=prec)
        assert "-4" in str(e.value)

"""The symmetric kernels Xi_X (COUPLE_XI output form).

App. A writes every coupling matrix as K^X_{l1 l2} = (2 l2 + 1) Xi_X(l1, l2);
the approximate pseudo-C_l covariance of Sec. 2 uses the same Xi evaluated on
the power spectrum of the squared mask.  With COUPLE_XI the entry points
write Xi itself:
* Xi is symmetric, exactly;
* K equals the float64 product (2 l2 + 1) * Xi bit for bit (same inputs and
  precision), for the full, band-limited, binned and batched forms;
* Xi matches the oracle's K / (2 l2 + 1) within the precision's tolerance;
* full sky (W_0 = 4 pi, W_l>0 = 0; mask^2 = mask = 1) gives the closed form
  Xi_TT = delta_{l1 l2} / (2 l1 + 1), and the same for EE, BB on l >= 2.
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
    c = couple.couple_init(1200)
    yield c
    couple.couple_free(c)


def _gpu(torch, arr):
    return torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64)).cuda()


def _windows(lmax, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.01, 2.0, 2 * lmax + 1) for _ in range(3)]


def _col_factor(torch, n):
    return (2.0 * torch.arange(n, dtype=torch.float64, device="cuda") + 1.0)[None, None, :]


@pytest.mark.parametrize("lmax", [0, 2, 65, 257, 1100])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_xi_symmetric_and_k_is_its_product(torch_gpu, ctx, lmax, precision):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    _say("xi lmax=%d %s" % (lmax, precision))
    dW = [_gpu(torch, w) for w in _windows(lmax, 40 + lmax)]
    X = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision, xi=True)
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision)
    assert torch.equal(X, X.transpose(1, 2))
    assert torch.equal(K, _col_factor(torch, lmax + 1) * X)
    assert torch.equal(X[2], X[3])
    del X, K


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
def test_xi_against_oracle(torch_gpu, ctx, oracle_bulk, precision, tol):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 300
    Ws = _windows(lmax, 9)
    dW = [_gpu(torch, w) for w in Ws]
    X = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision, xi=True).cpu().numpy()
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, spectra=SPEC5)
    f = 2.0 * np.arange(lmax + 1) + 1.0
    for i, s in enumerate(SPEC5):
        assert_parity(X[i], Kr[i] / f[None, :], Ar[i] / f[None, :], tol, "Xi %s %s" % (s, precision))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_xi_full_sky_closed_form(torch_gpu, ctx, precision):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 400
    w = np.zeros(2 * lmax + 1)
    w[0] = 4 * math.pi
    dw = _gpu(torch, w)
    X = couple.couple_matrix(ctx, dw, dw, dw, lmax, spectra=("TT", "TE", "EE", "BB"), precision=precision,
                             xi=True).cpu().numpy()
    l = np.arange(lmax + 1)
    ref = np.diag(1.0 / (2 * l + 1.0))
    tol = TOL_FP64 if precision == "fp64" else TOL_FP32C
    for i in range(4):
        r = ref.copy()
        if i > 0:
            r[:2, :2] = 0.0
        nz = r != 0
        assert np.max(np.abs(X[i][nz] - r[nz]) / r[nz]) < tol
        assert np.all(X[i][~nz] == 0.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_xi_band_and_bins(torch_gpu, ctx, precision):
    """Band-limited Xi, and binned Xi = the bin operator applied to Xi; K of
    the same band is (2 l2 + 1) Xi bit for bit."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax, lo, hi = 600, 4, 180
    dW = [_gpu(torch, w) for w in _windows(lmax, 3)]
    spectra = ("TT", "EE", "EB")
    X = couple.couple_band(ctx, lo, hi, *dW, lmax, spectra=spectra, precision=precision, xi=True)
    K = couple.couple_band(ctx, lo, hi, *dW, lmax, spectra=spectra, precision=precision)
    assert torch.equal(X, X.transpose(1, 2))
    assert torch.equal(K, _col_factor(torch, lmax + 1) * X)
    edges = [0, 2, 40, 41, 300, 301, 601]
    Xb = couple.couple_band(ctx, lo, hi, *dW, lmax, spectra=spectra, precision=precision, xi=True,
                            bin_edges=edges).cpu().numpy()
    Xf = X.cpu().numpy()
    for b in range(len(edges) - 1):
        for c in range(len(edges) - 1):
            blk = Xf[:, edges[b]:edges[b + 1], edges[c]:edges[c + 1]]
            ref = blk.sum(axis=(1, 2)) / (edges[b + 1] - edges[b])
            assert np.allclose(Xb[:, b, c], ref, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("precision", ["mfma_fp32", "mfma_bf16x3", "fp32c"])
def test_xi_batched(torch_gpu, ctx, precision):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmaxes = [200, 77, 130]
    Ws = [_windows(L, 500 + L) for L in lmaxes]
    dW = [[_gpu(torch, w[s]) for w in Ws] for s in range(3)]
    couple.couple_reserve_batched(ctx, lmaxes)
    X = couple.couple_matrix_batched(ctx, lmaxes, *dW, precision=precision, xi=True)
    K = couple.couple_matrix_batched(ctx, lmaxes, *dW, precision=precision)
    for m, L in enumerate(lmaxes):
        assert torch.equal(X[m], X[m].transpose(1, 2)), m
        assert torch.equal(K[m], _col_factor(torch, L + 1) * X[m]), m
    Xb = couple.couple_band_batched(ctx, 0, 400, [dW[0][0]], None, [dW[2][0]], 200, spectra=("TT", "EE"),
                                    precision="fp64", xi=True)
    Kb = couple.couple_band_batched(ctx, 0, 400, [dW[0][0]], None, [dW[2][0]], 200, spectra=("TT", "EE"),
                                    precision="fp64")
    assert torch.equal(Kb, _col_factor(torch, 201)[None] * Xb)

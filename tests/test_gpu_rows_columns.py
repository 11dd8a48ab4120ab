"""couple_matrix beyond the small full-matrix cases.

* couple_band over the whole l3 range [0, 2 lmax] is the same operation as
  couple_matrix: the two entry points agree bit for bit, over ragged sizes
  up to lmax = 2600.
* Whole rows and whole columns (both triangles, K_{l1 l2} = (2 l2 + 1) Xi and
  K_{l2 l1} = (2 l1 + 1) Xi) at strip-block and fill-tile edges against the
  oracle at lmax = 1100.
* Graph capture at lmax = 1100, and back-to-back calls on a caller's stream.
"""
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
    c = couple.couple_init(2600)
    yield c
    couple.couple_free(c)


def _gpu(torch, arr):
    return torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64)).cuda()


def _windows(lmax, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.01, 2.0, 2 * lmax + 1) for _ in range(3)]


@pytest.mark.parametrize("lmax", [0, 1, 2, 63, 64, 65, 255, 256, 257, 1100, 2600])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_matrix_equals_full_band(torch_gpu, ctx, lmax, precision):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    _say("couple_matrix vs couple_band [0, 2 lmax] lmax=%d %s" % (lmax, precision))
    dW = [_gpu(torch, w) for w in _windows(lmax, 90 + lmax)]
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision)
    Kb = couple.couple_band(ctx, 0, 2 * lmax, *dW, lmax, spectra=SPEC5, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(K, Kb)
    del K, Kb


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32c", TOL_FP32C)])
def test_rows_and_columns(torch_gpu, ctx, oracle_bulk, precision, tol):
    """Whole rows and columns (both triangles) at block and tile edges, against
    the oracle."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 1100
    Ws = _windows(lmax, 5)
    dW = [_gpu(torch, w) for w in Ws]
    rows = np.array(sorted({0, 1, 2, 63, 64, 255, 256, 257, 511, 512, 700, lmax - 256, lmax - 1, lmax}))
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision)
    got = K[:, torch.as_tensor(rows).cuda(), :].cpu().numpy()
    cols = K[:, :, torch.as_tensor(rows).cuda()].cpu().numpy()
    del K
    Kr, Ar = oracle_bulk.coupling_rows(lmax, *Ws, rows=rows, spectra=SPEC5)
    for i, s in enumerate(SPEC5):
        assert_parity(got[i], Kr[i], Ar[i], tol, "%s %s rows" % (precision, s))
        # columns: K_{l1 l2} = (2 l2 + 1) Xi(l1, l2), so K[:, r] = (2r+1)/(2l+1) K[r, :]
        l = np.arange(lmax + 1)
        ref_c = (Kr[i] * ((2 * rows[:, None] + 1.0) / (2 * l[None, :] + 1.0))).T
        abs_c = (Ar[i] * ((2 * rows[:, None] + 1.0) / (2 * l[None, :] + 1.0))).T
        assert_parity(cols[i], ref_c, abs_c, tol, "%s %s columns" % (precision, s))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_graph_replay_lmax1100(torch_gpu, ctx, precision):
    """The call enqueues kernels only: replays of a captured graph reproduce the
    eager result, with eager work and synchronisations in between."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 1100
    dW = [_gpu(torch, w) for w in _windows(lmax, 77)]
    eager = couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision).clone()
    out = torch.empty_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        couple.couple_matrix(ctx, *dW, lmax, spectra=SPEC5, precision=precision, out=out)
    for rep in range(4):
        out.fill_(float("nan"))
        x = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del x
    del graph


def test_back_to_back_on_callers_stream(torch_gpu, ctx):
    """Two calls queued back to back on a caller's stream, each followed by a
    copy of its output on the same stream, give the results of separate calls."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lmax = 2600
    dA = [_gpu(torch, w) for w in _windows(lmax, 1)]
    dB = [_gpu(torch, w) for w in _windows(lmax, 2)]
    refA = couple.couple_matrix(ctx, *dA, lmax, spectra=("TT", "EE"), precision="fp32c").clone()
    refB = couple.couple_matrix(ctx, *dB, lmax, spectra=("TT", "EE"), precision="fp32c").clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        outA = torch.full_like(refA, float("nan"))
        outB = torch.full_like(refB, float("nan"))
        couple.couple_matrix(ctx, *dA, lmax, spectra=("TT", "EE"), precision="fp32c", out=outA)
        copyA = outA.clone()
        couple.couple_matrix(ctx, *dB, lmax, spectra=("TT", "EE"), precision="fp32c", out=outB)
        copyB = outB.clone()
    s.synchronize()
    assert torch.equal(copyA, refA)
    assert torch.equal(copyB, refB)
    assert torch.equal(outA, refA)

"""The binned MASTER solve on the GPU (couple_bin_spectra, couple_master_solve)
against the oracle (oracle/master.py, numpy's LAPACK solve).

* Binning of pseudo-spectra, ragged bins, more than 512 bins (staged edges).
* Random TT and E/B block systems, one and several right-hand sides, a system
  that needs row exchanges: agreement with numpy within a bound from the
  condition number; systems of 6000 to 9000 unknowns by their backward error.
* A singular system gives NaN (small, 100 unknowns on one work-group, 700
  through the multi-work-group path and its tall panels); argument errors are
  caught on the host.
* End to end: windows -> binned K (couple_band) -> pseudo-spectra of a C_l
  that is constant inside each bin -> solve.  For such a C_l the binned
  relation of Sec. 2 eq. pseudo_cl is exact, so the solve must return the
  bin values of C_l; the oracle's own chain (oracle K, binned, LAPACK)
  agrees with it.
* One captured graph of bin + solve replays to the eager result, on both paths.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _system(n, rng):
    return np.eye(n) + 0.3 * rng.standard_normal((n, n)) / math.sqrt(n)


def _check_solution(x, A, b, what):
    """|x - x_ref| <= 64 cond(A) eps |x_ref| (backward-stable solves)."""
    ref = np.linalg.solve(A, b.T).T
    bound = 64 * np.linalg.cond(A) * np.finfo(float).eps * np.max(np.abs(ref))
    err = np.max(np.abs(x - ref))
    assert err <= bound, (what, err, bound)
    return err


@pytest.mark.parametrize("n_bins,width", [(7, None), (600, 1)])
def test_bin_spectra(torch_gpu, ctx, n_bins, width):
    from paper_2602_15605_amd import couple
    from oracle import master
    torch = torch_gpu
    rng = np.random.default_rng(n_bins)
    if width is None:
        edges = [0, 1, 2, 40, 41, 300, 301, 700]
    else:
        edges = list(range(5, 5 + n_bins + 1))
    cl = rng.uniform(0.1, 3.0, (3, 701))
    got = couple.couple_bin_spectra(ctx, _gpu(torch, cl), edges).cpu().numpy()
    ref = master.bin_spectrum(cl, edges)
    assert np.allclose(got, ref, rtol=1e-14, atol=0)
    one = couple.couple_bin_spectra(ctx, _gpu(torch, cl[1]), edges).cpu().numpy()
    assert np.array_equal(one, got[1])


@pytest.mark.parametrize("n,n_rhs", [(1, 1), (2, 1), (63, 1), (64, 3), (65, 1), (200, 2), (399, 1), (400, 1), (401, 2),
                                     (1023, 1), (2049, 3), (4000, 96)])
def test_solve_tt_random(torch_gpu, ctx, n, n_rhs):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    _say("solve TT n=%d n_rhs=%d" % (n, n_rhs))
    rng = np.random.default_rng(n)
    A = _system(n, rng)
    b = rng.standard_normal((n_rhs, n))
    x = couple.couple_master_solve(ctx, _gpu(torch, A), _gpu(torch, b)).cpu().numpy()
    err = _check_solution(x, A, b, "TT n=%d" % n)
    _say("  max abs err %.2e" % err)


@pytest.mark.parametrize("n,pol", [(6000, False), (9000, False), (3100, True)])
def test_solve_large(torch_gpu, ctx, n, pol):
    """Systems beyond 4096 unknowns, whose first panels are factorised 2 (over
    4096 rows) and 1 (over 8192 rows) columns at a time: the backward error
    |A x - b| / (|A| |x|) within 64 m eps (a condition number costs too much
    here), and the solution against LAPACK where that is affordable."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    m = 2 * n if pol else n
    _say("solve large m=%d" % m)
    rng = np.random.default_rng(m)
    if pol:
        K3 = np.stack([_system(n, rng), _system(n, rng), 0.05 * rng.standard_normal((n, n))])
        A = np.block([[K3[0], K3[2]], [K3[2], K3[1]]])
        Kg = _gpu(torch, K3)
    else:
        A = _system(n, rng)
        Kg = _gpu(torch, A)
    b = rng.standard_normal(m)
    x = couple.couple_master_solve(ctx, Kg, _gpu(torch, b), pol=pol).cpu().numpy()
    assert np.all(np.isfinite(x))
    r = np.abs(A @ x - b).max()
    berr = r / (np.abs(A).sum(axis=1).max() * np.abs(x).max())
    _say("  backward error %.2e" % berr)
    assert berr <= 64 * m * np.finfo(float).eps
    if m <= 6200:
        ref = np.linalg.solve(A, b)
        assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("n,n_rhs", [(1, 1), (31, 2), (200, 1), (1000, 4)])
def test_solve_pol_random(torch_gpu, ctx, n, n_rhs):
    from paper_2602_15605_amd import couple
    from oracle import master
    torch = torch_gpu
    rng = np.random.default_rng(100 + n)
    Kee, Kbb = _system(n, rng), _system(n, rng)
    Keb = 0.05 * rng.standard_normal((n, n))
    ct = rng.standard_normal((n_rhs, 2 * n))
    K3 = np.stack([Kee, Kbb, Keb])
    x = couple.couple_master_solve(ctx, _gpu(torch, K3), _gpu(torch, ct), pol=True).cpu().numpy()
    ee, bb = master.solve_pol(Kee, Kbb, Keb, ct[:, :n], ct[:, n:])
    A = np.block([[Kee, Keb], [Keb, Kbb]])
    bound = 64 * np.linalg.cond(A) * np.finfo(float).eps * max(np.max(np.abs(ee)), np.max(np.abs(bb)))
    assert np.max(np.abs(x[:, :n] - ee)) <= bound
    assert np.max(np.abs(x[:, n:] - bb)) <= bound


@pytest.mark.parametrize("n", [50, 450])
def test_solve_needs_row_exchanges(torch_gpu, ctx, n):
    """A permutation matrix has zeros on the diagonal: elimination without row
    exchanges would divide by zero; with them the solution is exact (one
    work-group at 50 unknowns, the multi-work-group path at 450)."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    perm = np.random.default_rng(5).permutation(n)
    while np.any(perm == np.arange(n)):
        perm = np.random.default_rng(int(perm[0]) + 7).permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 2.0
    b = np.arange(1.0, n + 1.0)
    x = couple.couple_master_solve(ctx, _gpu(torch, P), _gpu(torch, b)).cpu().numpy()
    ref = np.zeros(n)
    ref[perm] = b / 2.0
    assert np.array_equal(x, ref)


def test_singular_system_gives_nan(torch_gpu, ctx):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    A = np.ones((6, 6))
    x = couple.couple_master_solve(ctx, _gpu(torch, A), _gpu(torch, np.arange(6.0))).cpu().numpy()
    assert np.all(np.isnan(x))
    Z = np.zeros((3, 4, 4))
    x = couple.couple_master_solve(ctx, _gpu(torch, Z), _gpu(torch, np.ones((2, 8))), pol=True).cpu().numpy()
    assert x.shape == (2, 8) and np.all(np.isnan(x))
    # a good system on the same context right after
    x = couple.couple_master_solve(ctx, _gpu(torch, 4.0 * np.eye(3)), _gpu(torch, np.ones(3))).cpu().numpy()
    assert np.array_equal(x, np.full(3, 0.25))


def test_singular_tall_system_gives_nan(torch_gpu, ctx):
    """Singular systems of 100 and 700 unknowns give NaN.

    * 100 unknowns (one work-group): two equal rows.  Both get the same
      updates, so when one becomes a pivot the other is reduced to exact zeros
      and a later pivot column is zero.
    * 700 unknowns (outer panels spread over the chip): a zero column.  Every
      update subtracts multiples of that column's U entries, which are zero,
      so it stays exactly zero under any blocking; placed at 3 it is met in a
      panel taller than one wave handles, at 650 in a short one.  (Equal rows
      are not used here: the blocked update sums a row's multipliers in
      another order than the pivot row's own elimination, so the difference
      is rounding-sized, not zero.)
    """
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    rng = np.random.default_rng(700)
    A = _system(100, rng)
    A[90] = A[10]
    x = couple.couple_master_solve(ctx, _gpu(torch, A), _gpu(torch, rng.standard_normal((2, 100)))).cpu().numpy()
    assert x.shape == (2, 100) and np.all(np.isnan(x))
    for col in (3, 650):
        A = _system(700, rng)
        A[:, col] = 0.0
        x = couple.couple_master_solve(ctx, _gpu(torch, A), _gpu(torch, rng.standard_normal((2, 700)))).cpu().numpy()
        assert x.shape == (2, 700) and np.all(np.isnan(x)), col
    # a system of the same size right after solves (the flag is cleared)
    A = _system(700, np.random.default_rng(701))
    b = rng.standard_normal(700)
    x = couple.couple_master_solve(ctx, _gpu(torch, A), _gpu(torch, b)).cpu().numpy()
    _check_solution(x, A, b, "700 after singular")


def test_argument_errors(torch_gpu, ctx):
    import ctypes
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    lib = couple.load_library()
    t = _gpu(torch, np.ones(16))
    p = ctypes.c_void_p(t.data_ptr())
    h = ctx.handle
    assert lib.couple_master_solve(h, 2, 4, p, 1, p, p, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_master_solve(h, 0, 0, p, 1, p, p, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_master_solve(h, 0, 4, p, 0, p, p, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_master_solve(h, 0, 15840, p, 1, p, p, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_master_solve(h, 1, 7920, p, 1, p, p, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_master_solve(h, 0, 15000, p, 841, p, p, p, None) == couple.COUPLE_EINVAL
    assert "exceed" in couple.couple_last_error(ctx)
    assert lib.couple_master_solve(h, 0, 4, None, 1, p, p, p, None) == couple.COUPLE_EINVAL
    odd = ctypes.c_void_p(t.data_ptr() + 4)
    assert lib.couple_master_solve(h, 0, 4, odd, 1, p, p, p, None) == couple.COUPLE_EINVAL
    edges = (ctypes.c_int * 3)(0, 5, 5)
    assert lib.couple_bin_spectra(h, 1, p, 16, edges, 2, p, None) == couple.COUPLE_EINVAL
    edges = (ctypes.c_int * 3)(0, 5, 17)
    assert lib.couple_bin_spectra(h, 1, p, 16, edges, 2, p, None) == couple.COUPLE_EINVAL
    assert lib.couple_bin_spectra(h, 0, p, 16, edges, 2, p, None) == couple.COUPLE_EINVAL


def _piecewise(edges, values, length):
    c = np.zeros(length)
    for b in range(len(edges) - 1):
        c[edges[b]:edges[b + 1]] = values[b]
    return c


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_master_end_to_end(torch_gpu, ctx, oracle_bulk, precision):
    from paper_2602_15605_amd import couple, synth
    from oracle import master
    torch = torch_gpu
    lmax = 300
    W = [synth.window_spectrum(lmax, 120.0, 8800 + s) for s in range(3)]
    dW = [_gpu(torch, w) for w in W]
    rng = np.random.default_rng(11)
    # TT: bins of 10 from l = 0
    e_tt = list(range(0, lmax + 2, 10))
    if e_tt[-1] != lmax + 1:
        e_tt.append(lmax + 1)
    nb = len(e_tt) - 1
    c_tt = rng.uniform(0.5, 2.0, nb)
    Kr, _ = oracle_bulk.coupling_rows(lmax, *W, spectra=("TT", "EE", "BB", "EB"))
    ct_l = Kr[0] @ _piecewise(e_tt, c_tt, lmax + 1)            # <C~^TT> of Sec. 2 for this C^TT
    Kb = couple.couple_band(ctx, 0, 2 * lmax, dW[0], None, None, lmax, spectra=("TT",), precision=precision,
                            bin_edges=e_tt)
    ctb = couple.couple_bin_spectra(ctx, _gpu(torch, ct_l), e_tt)
    x = couple.couple_master_solve(ctx, Kb[0].contiguous(), ctb).cpu().numpy()
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert np.max(np.abs(x - c_tt) / c_tt) < tol, np.max(np.abs(x - c_tt) / c_tt)
    xo = master.solve_tt(master.bin_matrix(Kr[0], e_tt), master.bin_spectrum(ct_l, e_tt))
    assert np.max(np.abs(x - xo) / c_tt) < tol
    # E/B: bins from l = 2 (polarization rows 0 and 1 vanish)
    e_p = list(range(2, lmax + 2, 12))
    if e_p[-1] != lmax + 1:
        e_p.append(lmax + 1)
    nb = len(e_p) - 1
    c_ee, c_bb = rng.uniform(0.5, 2.0, nb), rng.uniform(0.05, 0.2, nb)
    pe, pb = _piecewise(e_p, c_ee, lmax + 1), _piecewise(e_p, c_bb, lmax + 1)
    ct_ee = Kr[1] @ pe + Kr[3] @ pb
    ct_bb = Kr[3] @ pe + Kr[2] @ pb
    K3 = couple.couple_band(ctx, 0, 2 * lmax, None, None, dW[2], lmax, spectra=("EE", "BB", "EB"),
                            precision=precision, bin_edges=e_p)
    rhs = couple.couple_bin_spectra(ctx, _gpu(torch, np.stack([ct_ee, ct_bb])), e_p).reshape(-1)
    x = couple.couple_master_solve(ctx, K3, rhs, pol=True).cpu().numpy()
    assert np.max(np.abs(x[:nb] - c_ee) / c_ee) < tol
    assert np.max(np.abs(x[nb:] - c_bb) / c_bb) < 10 * tol
    _say("E/B end to end %s: max rel err EE %.2e BB %.2e" % (
        precision, np.max(np.abs(x[:nb] - c_ee) / c_ee), np.max(np.abs(x[nb:] - c_bb) / c_bb)))


@pytest.mark.parametrize("n,pol", [(120, False), (300, True)])
def test_graph_replay(torch_gpu, ctx, n, pol):
    """One launch for 120 unknowns (TT); the multi-work-group sequence for the
    600-unknown E/B block.  Up to 512 bins the binning is capturable too."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    rng = np.random.default_rng(3)
    m = 2 * n if pol else n
    K = _gpu(torch, np.stack([_system(n, rng), _system(n, rng), 0.05 * rng.standard_normal((n, n))])
             if pol else _system(n, rng))
    ns = 2 if pol else 1
    cl = _gpu(torch, rng.uniform(0.5, 1.5, (ns, 3 * n)))
    edges = list(range(0, 3 * n + 1, 3))
    work = torch.empty(m * (m + 1), dtype=torch.float64, device="cuda")
    ctb = torch.empty((ns, n), dtype=torch.float64, device="cuda")
    x = torch.empty((1, m), dtype=torch.float64, device="cuda")

    def call():
        couple.couple_bin_spectra(ctx, cl, edges, out=ctb)
        couple.couple_master_solve(ctx, K, ctb.reshape(1, -1), pol=pol, work=work, out=x)

    call()
    torch.cuda.synchronize()
    eager = x.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for rep in range(3):
        x.fill_(float("nan"))
        ctb.fill_(float("nan"))
        y = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, eager), rep
        del y
    del graph


def test_binding_rejects_small_buffers(torch_gpu, ctx):
    """The C ABI cannot see the size of a caller's device buffer; the binding
    checks work and out before any launch."""
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    K = _gpu(torch, np.eye(10))
    b = _gpu(torch, np.ones(10))
    with pytest.raises(couple.CoupleError, match="work"):
        couple.couple_master_solve(ctx, K, b, work=torch.empty(50, dtype=torch.float64, device="cuda"))
    with pytest.raises(couple.CoupleError, match="out"):
        couple.couple_master_solve(ctx, K, b, out=torch.empty(5, dtype=torch.float64, device="cuda"))
    with pytest.raises(couple.CoupleError, match="expected"):
        couple.couple_master_solve(ctx, K, _gpu(torch, np.ones(20)), pol=True)
    with pytest.raises(couple.CoupleError, match="out"):
        couple.couple_bin_spectra(ctx, _gpu(torch, np.ones((2, 30))), [0, 10, 30],
                                  out=torch.empty(3, dtype=torch.float64, device="cuda"))
    with pytest.raises(couple.CoupleError, match="out"):
        couple.couple_threej_rows(ctx, [5, 6], [5, 6], 0, stride=13,
                                  out=torch.empty(20, dtype=torch.float64, device="cuda"))
    with pytest.raises(couple.CoupleError, match="too small"):
        couple.couple_band(ctx, 0, 20, b, None, None, 9, spectra=("TT",),
                           out=torch.empty(50, dtype=torch.float64, device="cuda"))

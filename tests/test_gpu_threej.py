"""Rows of 3j symbols (l1 l2 l3; -m m 0), m = 0, 1, 2, from the tables on the
GPU (couple_threej_rows) against the oracle's Schulten--Gordon rows (long
double, pinned to exact Racah values in tests/test_oracle_bulk.py).

* every pair l1, l2 <= 40 and sampled pairs to l = 6000: max |got - ref| over
  a row within 1e-13 of the row's largest |ref|, and 1e-12 relative on the
  elements above 1e-3 of it;
* at l up to 16384 (the limit), the orthogonality sums the closed forms do
  not impose: sum (2 l3 + 1) f^2 = 1, its even-L half = 1/2 for m > 0, and
  rows of different m orthogonal;
* pairs outside [0, lmax_max] give NaN rows; a short stride cuts rows.
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
    c = couple.couple_init(6000)
    yield c
    couple.couple_free(c)


def _check_rows(got, pairs, m, oracle_bulk, tag):
    worst = 0.0
    for p, (l1, l2) in enumerate(pairs):
        ref = oracle_bulk.threej_row(l1, l2, -m)
        n = len(ref)
        g = got[p, :n]
        big = np.max(np.abs(ref))
        if big == 0.0:
            assert np.all(g == 0.0), (tag, l1, l2)
            continue
        err = np.max(np.abs(g - ref)) / big
        assert err <= 1e-13, (tag, l1, l2, err)
        sel = np.abs(ref) > 1e-3 * big
        assert np.all(np.abs(g[sel] - ref[sel]) <= 1e-12 * np.abs(ref[sel])), (tag, l1, l2)
        assert np.all(got[p, n:] == 0.0)
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("m", [0, 1, 2])
def test_rows_small_all_pairs(torch_gpu, ctx, oracle_bulk, m):
    from paper_2602_15605_amd import couple
    pairs = [(l1, l2) for l1 in range(41) for l2 in range(41)]
    got = couple.couple_threej_rows(ctx, [p[0] for p in pairs], [p[1] for p in pairs], m).cpu().numpy()
    assert got.shape == (len(pairs), 81)
    worst = _check_rows(got, pairs, m, oracle_bulk, "small m=%d" % m)
    _say("m=%d all pairs <= 40: worst row error %.2e" % (m, worst))


@pytest.mark.parametrize("m", [0, 1, 2])
def test_rows_large_sampled(torch_gpu, ctx, oracle_bulk, m):
    from paper_2602_15605_amd import couple
    pairs = [(6000, 6000), (5999, 6000), (2, 6000), (1, 6000), (3001, 4444), (1234, 17), (4000, 3999),
             (6000, 0), (777, 778)]
    got = couple.couple_threej_rows(ctx, [p[0] for p in pairs], [p[1] for p in pairs], m).cpu().numpy()
    worst = _check_rows(got, pairs, m, oracle_bulk, "large m=%d" % m)
    _say("m=%d sampled pairs to 6000: worst row error %.2e" % (m, worst))


def test_orthogonality_at_the_limit(torch_gpu):
    from paper_2602_15605_amd import couple
    torch = torch_gpu
    L = couple.LMAX_LIMIT
    c = couple.couple_init(L)
    try:
        pairs = [(L, L), (L - 1, L), (2, L), (8191, 16000), (12345, 12346)]
        l1 = [p[0] for p in pairs]
        l2 = [p[1] for p in pairs]
        rows = [couple.couple_threej_rows(c, l1, l2, m).cpu().numpy() for m in (0, 1, 2)]
    finally:
        couple.couple_free(c)
    for p, (a, b) in enumerate(pairs):
        n = 2 * min(a, b) + 1
        l3 = np.arange(abs(a - b), a + b + 1)
        w = 2.0 * l3 + 1.0
        even = (a + b + l3) % 2 == 0
        x, y, z = (r[p, :n] for r in rows)
        for f in (x, y, z):
            assert math.fsum(w * f * f) == pytest.approx(1.0, abs=1e-12), (a, b)
        for f in (y, z):
            assert math.fsum((w * f * f)[even]) == pytest.approx(0.5, abs=1e-12), (a, b)
        assert abs(math.fsum(w * x * y)) < 1e-12 and abs(math.fsum(w * x * z)) < 1e-12
        assert abs(math.fsum(w * y * z)) < 1e-12


def test_invalid_pairs_and_short_stride(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import couple
    got = couple.couple_threej_rows(ctx, [10, -1, 6001, 3], [12, 5, 2, 6002], 2).cpu().numpy()
    assert np.all(np.isnan(got[1])) and np.all(np.isnan(got[2])) and np.all(np.isnan(got[3]))
    ref = oracle_bulk.threej_row(10, 12, -2)
    assert np.allclose(got[0, :len(ref)], ref, rtol=0, atol=1e-15)
    for m in (0, 1, 2):
        full = couple.couple_threej_rows(ctx, [300], [400], m).cpu().numpy()
        for stride in (50, 51):                  # even and odd row lengths
            short = couple.couple_threej_rows(ctx, [300], [400], m, stride=stride).cpu().numpy()
            assert short.shape == (1, stride) and np.array_equal(short[0], full[0, :stride]), (m, stride)
    with pytest.raises(couple.CoupleError):
        couple.couple_threej_rows(ctx, [1], [1], 3)

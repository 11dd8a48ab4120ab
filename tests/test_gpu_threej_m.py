"""Rows of (l1 l2 l3; m1 m2 -m1-m2) for the small-m families, (1 1 -2) and
(2 2 -4) among them, from the tables on the GPU (couple_threej_rows_m)
against the oracle's general Schulten--Gordon rows (long double, pinned to
exact Racah values in tests/test_symbol_families.py).

* every pair l1, l2 <= 30 and sampled pairs to l = 6000, for the families, their
  m-flips, permutations and mixed signs: max |got - ref| over a row within
  1e-13 of the row's largest |ref|, and 1e-12 relative on the elements above
  1e-3 of it; the corner l3 << l1 = l2 is in the sample;
* at l up to 16384 (the limit, where the exact numerators are largest): the
  oracle rows for three pairs, and the orthogonality sum (2 l3 + 1) f^2 = 1;
* the (-m m 0) rows agree with couple_threej_rows; pairs outside
  [0, lmax_max] give NaN rows; a short stride cuts rows; magnetic numbers
  outside the families are refused.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FAMILIES = [(1, 1), (2, 2), (-1, -1), (-2, -2), (1, 2), (2, 1), (2, -1), (-1, 2), (-1, -1), (4, -2), (-2, 4),
            (1, -3), (0, 2), (2, 0), (-2, 2), (0, 0)]


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


def _check_rows(got, pairs, m1, m2, oracle_bulk, tag):
    worst = 0.0
    for p, (l1, l2) in enumerate(pairs):
        ref = oracle_bulk.threej_row_m(l1, l2, m1, m2)
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


@pytest.mark.parametrize("m1,m2", FAMILIES)
def test_rows_small_all_pairs(torch_gpu, ctx, oracle_bulk, m1, m2):
    from paper_2602_15605_amd import couple
    pairs = [(l1, l2) for l1 in range(31) for l2 in range(31)]
    _say("family (%d %d %d): all pairs <= 30" % (m1, m2, -m1 - m2))
    got = couple.couple_threej_rows_m(ctx, [p[0] for p in pairs], [p[1] for p in pairs], m1, m2).cpu().numpy()
    assert got.shape == (len(pairs), 61)
    worst = _check_rows(got, pairs, m1, m2, oracle_bulk, "small (%d,%d)" % (m1, m2))
    _say("  worst row error %.2e" % worst)


LARGE = [(6000, 6000), (5999, 6000), (2, 6000), (4, 6000), (3001, 4444), (1234, 17), (4000, 3999), (6000, 5),
         (777, 778), (5000, 5004)]


@pytest.mark.parametrize("m1,m2", [(1, 1), (2, 2), (-2, -2), (2, 1), (2, -1), (4, -2), (0, 2)])
def test_rows_large_sampled(torch_gpu, ctx, oracle_bulk, m1, m2):
    from paper_2602_15605_amd import couple
    _say("family (%d %d %d): sampled pairs to 6000" % (m1, m2, -m1 - m2))
    got = couple.couple_threej_rows_m(ctx, [p[0] for p in LARGE], [p[1] for p in LARGE], m1, m2).cpu().numpy()
    worst = _check_rows(got, LARGE, m1, m2, oracle_bulk, "large (%d,%d)" % (m1, m2))
    _say("  worst row error %.2e" % worst)


def test_rows_at_the_limit(torch_gpu, oracle_bulk):
    from paper_2602_15605_amd import couple
    L = couple.LMAX_LIMIT
    c = couple.couple_init(L)
    pairs = [(L, L), (L - 1, L), (3, L), (8191, 16000), (12345, 12346)]
    try:
        _say("families at lmax %d" % L)
        rows = {m: couple.couple_threej_rows_m(c, [p[0] for p in pairs], [p[1] for p in pairs], *m).cpu().numpy()
                for m in [(1, 1), (2, 2), (2, -1)]}
    finally:
        couple.couple_free(c)
    for m, got in rows.items():
        _check_rows(got[:3], pairs[:3], m[0], m[1], oracle_bulk, "limit %s" % (m,))
        for p, (a, b) in enumerate(pairs):
            n = 2 * min(a, b) + 1
            l3 = np.arange(abs(a - b), a + b + 1)
            f = got[p, :n]
            assert math.fsum((2.0 * l3 + 1.0) * f * f) == pytest.approx(1.0, abs=1e-12), (m, a, b)


@pytest.mark.parametrize("m", [0, 1, 2])
def test_agrees_with_the_minus_m_m_0_rows(torch_gpu, ctx, m):
    from paper_2602_15605_amd import couple
    pairs = [(l1, l2) for l1 in range(0, 41, 3) for l2 in range(0, 41, 4)] + LARGE
    l1 = [p[0] for p in pairs]
    l2 = [p[1] for p in pairs]
    a = couple.couple_threej_rows(ctx, l1, l2, m).cpu().numpy()
    b = couple.couple_threej_rows_m(ctx, l1, l2, -m, m).cpu().numpy()
    for p in range(len(pairs)):
        big = np.max(np.abs(a[p]))
        assert np.max(np.abs(a[p] - b[p])) <= 1e-13 * max(big, 1e-300), (m, pairs[p])


def test_invalid_pairs_short_stride_and_refusals(torch_gpu, ctx, oracle_bulk):
    from paper_2602_15605_amd import couple
    got = couple.couple_threej_rows_m(ctx, [10, -1, 6001, 3], [12, 5, 2, 6002], 2, 2).cpu().numpy()
    assert np.all(np.isnan(got[1])) and np.all(np.isnan(got[2])) and np.all(np.isnan(got[3]))
    ref = oracle_bulk.threej_row_m(10, 12, 2, 2)
    assert np.allclose(got[0, :len(ref)], ref, rtol=0, atol=1e-15)
    full = couple.couple_threej_rows_m(ctx, [300], [400], 1, 1).cpu().numpy()
    for stride in (50, 51):
        short = couple.couple_threej_rows_m(ctx, [300], [400], 1, 1, stride=stride).cpu().numpy()
        assert short.shape == (1, stride) and np.array_equal(short[0], full[0, :stride]), stride
    for (m1, m2) in [(3, 0), (0, 3), (3, -3), (3, 3), (-3, -1), (5, -1)]:
        with pytest.raises(couple.CoupleError):
            couple.couple_threej_rows_m(ctx, [10], [10], m1, m2)

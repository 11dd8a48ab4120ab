"""Host-side pieces of bench.py (no GPU): the oracle row sample keeps the
longest rows, and the TE plain-error helper."""
import numpy as np

import bench


def test_bench_rows_keep_ends():
    for lmax, n in ((6000, 400), (6000, 60), (2000, 30)):
        rows = bench.bench_rows(lmax, n)
        assert len(rows) <= n and len(rows) >= n - 4
        assert {0, 1, 2, lmax} <= set(rows.tolist())
        assert np.all(np.diff(rows) > 0)


def test_te_plain_error():
    K_ref = np.array([1.0, -2.0, 1e-6, 0.0])
    A_ref = np.array([1.0, 3.0, 1.0, 0.0])
    K = np.array([1.0 + 1e-9, -2.0 - 4e-9, 1.0, 0.0])
    # the third element is below the 1e-3 floor and the fourth has A_ref = 0
    assert abs(bench.te_plain_error(K, K_ref, A_ref) - 2e-9) < 1e-15


def test_band_triples_brute_force():
    """The band-limited triple count the band roofline divides by: even-L
    (l1 <= l2 <= lmax, l3 <= cut) triples, against a direct count."""
    import bench

    def brute(L, cut):
        n = 0
        for l1 in range(L + 1):
            for l2 in range(l1, L + 1):
                for l3 in range(l2 - l1, min(l1 + l2, cut) + 1):
                    n += (l1 + l2 + l3) % 2 == 0
        return n

    for L, cut in ((10, 4), (20, 7), (15, 40), (30, 0), (25, 25)):
        assert bench.band_triples(L, cut) == brute(L, cut), (L, cut)
    assert bench.band_triples(12, 10 ** 6) == bench.triples(12)

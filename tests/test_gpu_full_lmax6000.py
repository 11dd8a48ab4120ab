"""Every element of the four 6001 x 6001 matrices of the lmax = 6000 workload
(TT, TE, EE, BB over all l1, l2; the synthetic l_c = 1500 windows) against the
oracle, in FP64 (1e-12) and FP32C (1e-6).

The oracle evaluates the upper triangle l2 >= l1 element by element (its
long-double recursion, every l3 of the triangle).  The lower triangle follows
from the definition: the symbols squared (and the TE product) are symmetric
under l1 <-> l2, so K_{l2 l1} = (2 l1 + 1)/(2 l2 + 1) K_{l1 l2}, and likewise
the sum of |terms| A that the error metric divides by.  Rows are split into
interleaved chunks of equal oracle work, one test per chunk, so progress shows
as the chunks finish.  Besides the error metric of tests/_parity.py, TE is
also checked by the plain relative error |dK|/|K_ref| on the elements with
|K_ref| >= 1e-3 A_ref.  With COUPLE_PARITY_REPORT set, the worst element of
every (precision, spectrum) is written there as JSON after the last chunk.
"""
import json
import os
import sys

import numpy as np
import pytest

from _parity import TOL_FP32C, TOL_FP64

pytestmark = pytest.mark.gpu

LMAX = 6000
SPEC4 = ("TT", "TE", "EE", "BB")
N_CHUNKS = 8
TOLS = {"fp64": TOL_FP64, "fp32c": TOL_FP32C}
# plain relative error on TE elements with |K_ref| >= TE_FLOOR A_ref: at most
# the condition-aware error times A_ref/|K_ref| <= 1/TE_FLOOR
TE_FLOOR = 1e-3

_worst = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full_k():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_15605_amd import couple, synth
    W = synth.workload_windows(2)
    ctx = couple.couple_init(LMAX)
    dW = [torch.as_tensor(w).cuda() for w in W]
    Ks = {}
    try:
        for prec in ("fp64", "fp32c"):
            _say("[full lmax6000] couple_matrix %s" % prec)
            K = couple.couple_matrix(ctx, *dW, LMAX, spectra=SPEC4, precision=prec)
            torch.cuda.synchronize()
            Ks[prec] = K.cpu().numpy()
            del K
    finally:
        couple.couple_free(ctx)
    torch.cuda.empty_cache()
    return W, Ks


def _note(prec, spec, kind, err, l1, l2):
    key = (prec, spec, kind)
    if err > _worst.get(key, (-1.0,))[0]:
        _worst[key] = (float(err), int(l1), int(l2))


def _check_half(prec, spec, K, Kr, Ar, l1s, l2s):
    """K, Kr, Ar: flat arrays of compared elements at (l1s, l2s)."""
    zero = Ar == 0
    assert np.all(K[zero] == 0.0), "%s %s: %d elements should be exactly 0" % (
        prec, spec, int(np.count_nonzero(K[zero] != 0.0)))
    nz = ~zero
    rel = np.abs(K[nz] - Kr[nz]) / Ar[nz]
    i = int(np.argmax(rel))
    err = float(rel[i])
    _note(prec, spec, "metric", err, l1s[nz][i], l2s[nz][i])
    if spec == "TE":
        big = nz & (np.abs(Kr) >= TE_FLOOR * Ar)
        plain = np.abs(K[big] - Kr[big]) / np.abs(Kr[big])
        j = int(np.argmax(plain))
        _note(prec, spec, "plain", float(plain[j]), l1s[big][j], l2s[big][j])
        assert plain[j] <= TOLS[prec] / TE_FLOOR
    return err


@pytest.mark.parametrize("chunk", range(N_CHUNKS))
def test_full_matrices_lmax6000(full_k, oracle_bulk, chunk):
    W, Ks = full_k
    rows = np.arange(chunk, LMAX + 1, N_CHUNKS, dtype=np.int32)
    _say("[full lmax6000] oracle chunk %d: %d rows" % (chunk, len(rows)))
    Kr, Ar = oracle_bulk.coupling_rows(LMAX, *W, rows=rows, spectra=SPEC4, upper=True)
    col = np.arange(LMAX + 1)
    upper = col[None, :] >= rows[:, None]                      # [rows, l2]
    r_idx, c_idx = np.nonzero(upper)
    l1s, l2s = rows[r_idx], col[c_idx]
    # K_{l2 l1} = (2 l1 + 1)/(2 l2 + 1) K_{l1 l2}
    f = (2.0 * l1s + 1.0) / (2.0 * l2s + 1.0)
    for prec, K in Ks.items():
        worst = 0.0
        for s, spec in enumerate(SPEC4):
            Kref = Kr[s][r_idx, c_idx]
            Aref = Ar[s][r_idx, c_idx]
            e_up = _check_half(prec, spec, K[s][l1s, l2s], Kref, Aref, l1s, l2s)
            e_lo = _check_half(prec, spec, K[s][l2s, l1s], Kref * f, Aref * f, l2s, l1s)
            worst = max(worst, e_up, e_lo)
            assert e_up <= TOLS[prec] and e_lo <= TOLS[prec], (prec, spec, e_up, e_lo)
        _say("[full lmax6000] chunk %d %s worst %.3e" % (chunk, prec, worst))
    if chunk == N_CHUNKS - 1:
        report = {"%s %s %s" % k: {"err": v[0], "l1": v[1], "l2": v[2]} for k, v in sorted(_worst.items())}
        _say(json.dumps(report))
        path = os.environ.get("COUPLE_PARITY_REPORT")
        if path:
            with open(path, "w") as fh:
                json.dump(report, fh, indent=1)

"""Every element of the largest mask's four matrices in the 32-mask batched
workload (lmax uniform in [500, 4000]) against the oracle, for the two
matrix-core forms and the per-mask FP32C loop of couple_matrix_batched.

The other masks of the call are checked on sampled rows in
tests/test_gpu_batched.py; this one shows that no row outside the sample
breaks the bound.  The oracle evaluates the upper triangle and the lower one
follows from K_{l2 l1} = (2 l1 + 1)/(2 l2 + 1) K_{l1 l2} (the squared symbols
and the TE product are symmetric under l1 <-> l2), as in
tests/test_gpu_full_lmax6000.py.  Rows are split into interleaved chunks so
progress shows as they finish.
"""
import sys

import numpy as np
import pytest

from _parity import TOL_BF16X3, TOL_FP32C

pytestmark = pytest.mark.gpu

SPEC4 = ("TT", "TE", "EE", "BB")
PRECISIONS = {"mfma_fp32": TOL_FP32C, "mfma_bf16x3": TOL_BF16X3, "fp32c": TOL_FP32C}
N_CHUNKS = 4
_worst = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def largest_mask():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_15605_amd import couple, synth
    lmaxes = [int(x) for x in synth.batched_lmaxes()]
    m = int(np.argmax(lmaxes))
    Ws = [synth.workload_windows(3, mask=i) for i in range(len(lmaxes))]
    ctx = couple.couple_init(max(lmaxes))
    Ks = {}
    try:
        dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
        couple.couple_reserve_batched(ctx, lmaxes)
        for prec in PRECISIONS:
            _say("[batched full] couple_matrix_batched %s, 32 masks" % prec)
            outs = couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], spectra=SPEC4, precision=prec)
            torch.cuda.synchronize()
            Ks[prec] = outs[m].cpu().numpy()
            del outs
            torch.cuda.empty_cache()
    finally:
        couple.couple_free(ctx)
    return lmaxes[m], Ws[m], Ks


@pytest.mark.parametrize("chunk", range(N_CHUNKS))
def test_largest_mask_every_element(largest_mask, oracle_bulk, chunk):
    L, W, Ks = largest_mask
    rows = np.arange(chunk, L + 1, N_CHUNKS, dtype=np.int32)
    _say("[batched full] lmax %d oracle chunk %d: %d rows" % (L, chunk, len(rows)))
    Kr, Ar = oracle_bulk.coupling_rows(L, *W, rows=rows, spectra=SPEC4, upper=True)
    col = np.arange(L + 1)
    r_idx, c_idx = np.nonzero(col[None, :] >= rows[:, None])
    l1s, l2s = rows[r_idx], col[c_idx]
    f = (2.0 * l1s + 1.0) / (2.0 * l2s + 1.0)
    for prec, K in Ks.items():
        for s, spec in enumerate(SPEC4):
            Kref, Aref = Kr[s][r_idx, c_idx], Ar[s][r_idx, c_idx]
            for (got, ref, aref, a1, a2) in ((K[s][l1s, l2s], Kref, Aref, l1s, l2s),
                                             (K[s][l2s, l1s], Kref * f, Aref * f, l2s, l1s)):
                zero = aref == 0
                assert np.all(got[zero] == 0.0), (prec, spec)
                rel = np.abs(got[~zero] - ref[~zero]) / aref[~zero]
                i = int(np.argmax(rel))
                key = (prec, spec)
                if rel[i] > _worst.get(key, (-1.0,))[0]:
                    _worst[key] = (float(rel[i]), int(a1[~zero][i]), int(a2[~zero][i]))
                assert rel[i] <= PRECISIONS[prec], (prec, spec, float(rel[i]), int(a1[~zero][i]), int(a2[~zero][i]))
    _say("[batched full] chunk %d: %s" % (chunk, {"%s %s" % k: "%.2e" % v[0] for k, v in sorted(_worst.items())}))
    if chunk == N_CHUNKS - 1:
        for k, v in sorted(_worst.items()):
            _say("[batched full] worst %s %s: %.3e at (%d, %d)" % (k[0], k[1], v[0], v[1], v[2]))

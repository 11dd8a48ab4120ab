"""Binned MASTER solve (TEST INFRASTRUCTURE ONLY).

Sec. 2, eq. pseudo_cl: the expected pseudo-spectra are linear in the true
spectra,

    <C~^TT> = K^TT C^TT
    <C~^EE> = K^EE C^EE + K^EB C^BB

and, by the structure App. A states (Xi_BB has the form of Xi_EE, and
Xi_BE = Xi_EB), the B-mode line

    <C~^BB> = K^EB C^EE + K^BB C^BB.

Binning (the rule of couple_band: uniform average over the row bin, sum over
the column bin, i.e. C_l taken constant inside a bin):

    K_{b b'} = (1/n_b) sum_{l1 in b} sum_{l2 in b'} K_{l1 l2}
    C~_b     = (1/n_b) sum_{l in b} C~_l

and the binned system K_{b b'} C_{b'} = C~_b is solved with LAPACK's LU
(numpy.linalg.solve), a library primitive used as one step.

Pinned by tests/test_oracle_master.py: round trips through the relations
above written as separate matrix products, the full-sky identity, and the
closed form of the binned flat-window K^TT.
"""
import numpy as np


def bin_spectrum(cl, edges):
    """C~_b = (1/n_b) sum_{l in b} C~_l over the last axis."""
    cl = np.asarray(cl, dtype=np.float64)
    out = []
    for b in range(len(edges) - 1):
        lo, hi = int(edges[b]), int(edges[b + 1])
        out.append(cl[..., lo:hi].sum(axis=-1) / (hi - lo))
    return np.stack(out, axis=-1)


def bin_matrix(K, edges):
    """K_{b b'} = (1/n_b) sum_{l1 in b} sum_{l2 in b'} K_{l1 l2} over the last two axes."""
    K = np.asarray(K, dtype=np.float64)
    nb = len(edges) - 1
    out = np.empty(K.shape[:-2] + (nb, nb))
    for b in range(nb):
        r0, r1 = int(edges[b]), int(edges[b + 1])
        for c in range(nb):
            c0, c1 = int(edges[c]), int(edges[c + 1])
            out[..., b, c] = K[..., r0:r1, c0:c1].sum(axis=(-2, -1)) / (r1 - r0)
    return out


def solve_tt(Kb, ct_b):
    """C_b from K^TT_{b b'} C_{b'} = C~_b (ct_b: [n] or [n_rhs, n])."""
    ct_b = np.asarray(ct_b, dtype=np.float64)
    if ct_b.ndim == 1:
        return np.linalg.solve(Kb, ct_b)
    return np.linalg.solve(Kb, ct_b.T).T


def solve_pol(Kb_ee, Kb_bb, Kb_eb, ct_ee, ct_bb):
    """(C^EE_b, C^BB_b) from the E/B block system of eq. pseudo_cl, binned."""
    A = np.block([[Kb_ee, Kb_eb], [Kb_eb, Kb_bb]])
    n = Kb_ee.shape[0]
    rhs = np.concatenate([np.asarray(ct_ee, dtype=np.float64), np.asarray(ct_bb, dtype=np.float64)], axis=-1)
    if rhs.ndim == 1:
        x = np.linalg.solve(A, rhs)
    else:
        x = np.linalg.solve(A, rhs.T).T
    return x[..., :n], x[..., n:]

"""SVD truncation of the two-site wavefunction (oracle; test infrastructure).

After each update the paper's DMRG factorises the optimised two-site tensor
and keeps D states (Introduction: "matrix factorization"; Numerical
procedure: D controls the accuracy).  With U(1)xU(1) symmetry the
wavefunction is block diagonal in the enlarged-left sector, so:

  * each block Psi[q, Q-q] is decomposed separately (LAPACK gesdd);
  * all singular values are pooled and sorted descending, ties broken by
    (sector index, position inside the sector);
  * at most `max_keep` values strictly above `cutoff` are kept;
  * the truncation error is the sum of the discarded sigma^2.

By Eckart-Young the kept blocks give the best rank-restricted approximation
and ||Psi - Psi_kept||_F^2 equals the truncation error.
"""
from __future__ import annotations

import numpy as np

from .heff import Layout


def svd_truncate(lay: Layout, psi, max_keep: int, cutoff: float = 0.0):
    psi = np.asarray(psi, dtype=np.float64)
    dec = {}
    pool = []
    for a in lay.partner:
        U, S, Vt = np.linalg.svd(lay.block(psi, a), full_matrices=False)
        dec[a] = (U, S, Vt)
        for k, s in enumerate(S):
            pool.append((-s, a, k))
    pool.sort()
    kept = {a: 0 for a in dec}
    n = 0
    err = 0.0
    for (ms, a, k) in pool:
        s = -ms
        if n < max_keep and s > cutoff:
            kept[a] += 1
            n += 1
        else:
            err += s * s
    out = {}
    for a, (U, S, Vt) in dec.items():
        k = kept[a]
        out[a] = (U[:, :k], S[:k], Vt[:k, :])
    return out, err


def reconstruct(lay: Layout, parts):
    y = np.zeros(lay.total)
    for a, (U, S, Vt) in parts.items():
        lay.block(y, a)[...] = (U * S) @ Vt
    return y

"""Davidson eigensolver for the lowest eigenpair (oracle; test infrastructure).

The paper solves each DMRG update's hermitian eigenproblem with Lanczos or
Davidson (Numerical procedure section).  This is the standard Davidson
method (E. R. Davidson, J. Comput. Phys. 17, 87 (1975)) in the form the
project fixes:

  * start from the given vector (or the unit vector at argmin of the
    diagonal), normalised;
  * subspace V with W = H V; projected matrix G = V^T W, Ritz pair
    (theta, s) lowest eigenpair of G (dense eigh);
  * x = V s, residual r = W s - theta x; stop when ||r||_2 <= tol;
  * correction t = r / (theta - d) with |theta - d| clamped to >= 1e-8
    (sign kept), d the diagonal of H;
  * classical Gram-Schmidt of t against V, done twice (DGKS); t is dropped
    (and the iteration counts as stalled) if its norm falls below 1e-10;
  * when V holds max_subspace vectors, restart from the `restart_keep`
    lowest Ritz vectors.
"""
from __future__ import annotations

import numpy as np


def davidson(matvec, diag, x0=None, tol=1e-8, max_iter=200, max_subspace=24,
             restart_keep=2):
    d = np.asarray(diag, dtype=np.float64)
    n = d.size
    if x0 is None:
        x0 = np.zeros(n)
        x0[int(np.argmin(d))] = 1.0
    v = np.asarray(x0, dtype=np.float64).copy()
    v /= np.linalg.norm(v)
    V = [v]
    W = [matvec(v)]
    n_mv = 1
    theta, x, res = None, v, np.inf
    for it in range(1, max_iter + 1):
        Vm = np.stack(V, axis=1)
        Wm = np.stack(W, axis=1)
        G = Vm.T @ Wm
        G = 0.5 * (G + G.T)
        evals, evecs = np.linalg.eigh(G)
        theta = float(evals[0])
        s = evecs[:, 0]
        x = Vm @ s
        hx = Wm @ s
        r = hx - theta * x
        res = float(np.linalg.norm(r))
        if res <= tol:
            return dict(energy=theta, x=x, residual=res, iters=it, matvecs=n_mv, converged=True)
        if len(V) >= max_subspace:
            keep = evecs[:, :restart_keep]
            V = list((Vm @ keep).T)
            W = list((Wm @ keep).T)
            Vm = np.stack(V, axis=1)
        denom = theta - d
        small = np.abs(denom) < 1e-8
        denom = np.where(small, np.where(denom < 0, -1e-8, 1e-8), denom)
        t = r / denom
        for _ in range(2):
            t = t - Vm @ (Vm.T @ t)
        nt = np.linalg.norm(t)
        if nt < 1e-10:
            return dict(energy=theta, x=x, residual=res, iters=it, matvecs=n_mv, converged=False)
        t = t / nt
        V.append(t)
        W.append(matvec(t))
        n_mv += 1
    return dict(energy=theta, x=x, residual=res, iters=max_iter, matvecs=n_mv, converged=False)

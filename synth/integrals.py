"""Seeded synthetic one- and two-electron integrals (input construction only).

The paper's molecular integrals are not available, so small synthetic
active spaces stand in for them:

* h is real symmetric: the upper triangle (i <= j, row-major order) is drawn
  i.i.d. N(0,1), multiplied by exp(-|i-j|/4) and mirrored;
* V_ijkl = (ij|kl) = sum_{r=1..8} L^r_ij L^r_kl with each L^r real symmetric
  (upper triangle i.i.d. N(0, 0.3^2), mirrored): a positive-semidefinite
  Cholesky-style sum of 8 rank-1 pair-space factors, which has the full
  8-fold permutational symmetry of real orbitals;
* numpy PCG64 (`default_rng(seed)`), drawing h first and then L^1..L^8.
"""
from __future__ import annotations

import numpy as np


def _sym_upper(rng, n, scale, decay=None):
    m = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            v = rng.standard_normal() * scale
            if decay is not None:
                v *= decay(i, j)
            m[i, j] = m[j, i] = v
    return m


def integrals(n_orb: int, seed: int, n_chol: int = 8, chol_sd: float = 0.3):
    rng = np.random.default_rng(seed)
    h = _sym_upper(rng, n_orb, 1.0, decay=lambda i, j: np.exp(-abs(i - j) / 4.0))
    V = np.zeros((n_orb,) * 4)
    for _ in range(n_chol):
        Lr = _sym_upper(rng, n_orb, chol_sd)
        V += np.einsum("ij,kl->ijkl", Lr, Lr)
    return h, V


def hubbard_dimer(t: float, U: float):
    """Two-orbital Hubbard model: h = [[0,-t],[-t,0]], (ii|ii) = U."""
    h = np.array([[0.0, -t], [-t, 0.0]])
    V = np.zeros((2, 2, 2, 2))
    V[0, 0, 0, 0] = V[1, 1, 1, 1] = U
    return h, V

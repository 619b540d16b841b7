"""Fermionic Fock-space operators, built bit by bit (oracle; test infrastructure).

Conventions (the paper's MPS of Eq. 1 uses 4 states per spatial orbital; the
ordering below is this project's documented reading):

* spin-orbital ("mode") index m = 2*i + s, with s = 0 for alpha (up) and
  s = 1 for beta (down): orbital-major, alpha before beta, orbital 0 first;
* a basis state is an integer x whose bit m is the occupation n_m, and
  |x> = (a+_0)^{n_0} (a+_1)^{n_1} ... |vac>, so that
  a_m |x> = (-1)^{sum_{p<m} n_p} |x - 2^m| when n_m = 1 (Jordan-Wigner);
* one orbital's 4 local states in index order n_up + 2 n_dn are
  |0>, |up>, |dn>, |updn> with |updn> = a+_up a+_dn |0>, carrying
  (N, 2Sz) = (0,0), (1,1), (1,-1), (2,0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mode(i: int, s: int) -> int:
    return 2 * i + s


def popcount(x: int) -> int:
    return bin(x).count("1")


def qn_of(x: int, n_modes: int):
    """(N, 2Sz) of basis state x."""
    na = sum((x >> (2 * i)) & 1 for i in range(n_modes // 2))
    nb = sum((x >> (2 * i + 1)) & 1 for i in range(n_modes // 2))
    return na + nb, na - nb


def annihilator(m: int, n_modes: int) -> sp.csr_matrix:
    """Matrix of a_m on the full 2^n_modes Fock space (sparse, exact)."""
    dim = 1 << n_modes
    x = np.arange(dim, dtype=np.int64)
    occ = ((x >> m) & 1).astype(bool)
    below = x & ((1 << m) - 1)
    parity = np.zeros(dim, dtype=np.int64)
    for p in range(m):
        parity += (below >> p) & 1
    cols = x[occ]
    rows = cols - (1 << m)
    vals = np.where(parity[occ] % 2 == 1, -1.0, 1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


class FockSpace:
    """All 2^n_modes states of n_orb spatial orbitals, with a_m and a+_m."""

    def __init__(self, n_orb: int):
        self.n_orb = n_orb
        self.n_modes = 2 * n_orb
        self.dim = 1 << self.n_modes
        self._a = [annihilator(m, self.n_modes) for m in range(self.n_modes)]
        self.qn = np.array([qn_of(x, self.n_modes) for x in range(self.dim)], dtype=np.int64)

    def a(self, i: int, s: int) -> sp.csr_matrix:
        return self._a[mode(i, s)]

    def cdag(self, i: int, s: int) -> sp.csr_matrix:
        return self._a[mode(i, s)].T.tocsr()

    def op(self, factors) -> sp.csr_matrix:
        """Product of factors [(dagger, i, s), ...] in the written order."""
        out = sp.identity(self.dim, format="csr")
        for (dag, i, s) in factors:
            f = self.cdag(i, s) if dag else self.a(i, s)
            out = out @ f
        return out.tocsr()

    def sector(self, n: int, two_sz: int) -> np.ndarray:
        return np.nonzero((self.qn[:, 0] == n) & (self.qn[:, 1] == two_sz))[0]

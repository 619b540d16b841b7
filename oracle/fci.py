"""Full configuration interaction for the ab initio Hamiltonian (oracle).

The paper minimises <Psi|H|Psi>/<Psi|Psi> over MPS (Eq. 2); with unlimited
bond dimension the minimum is the FCI ground-state energy, which this module
computes exactly.  H is the spin-free quantum-chemistry Hamiltonian

    H = sum_{pq,s} h_pq a+_ps a_qs
        + 1/2 sum_{pqrs,s,t} V_pqrs a+_ps a+_rt a_st a_qs,

V_pqrs = (pq|rs) in chemists' notation, real orbitals, no core energy.  It is
assembled from the spin-summed excitation operators E_pq = sum_s a+_ps a_qs
through the textbook identity
    sum_{s,t} a+_ps a+_rt a_st a_qs = E_pq E_rs - delta_qr E_ps,
inside one (N_alpha, N_beta) sector of the Fock space (oracle; test
infrastructure).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fock import FockSpace


def sector_basis(fs: FockSpace, n_a: int, n_b: int) -> np.ndarray:
    return fs.sector(n_a + n_b, n_a - n_b)


def excitation_ops(fs: FockSpace, idx: np.ndarray):
    """E_pq restricted to the states idx (sparse, exact)."""
    n = fs.n_orb
    E = [[None] * n for _ in range(n)]
    for p in range(n):
        for q in range(n):
            full = fs.cdag(p, 0) @ fs.a(q, 0) + fs.cdag(p, 1) @ fs.a(q, 1)
            E[p][q] = full.tocsr()[idx][:, idx].tocsr()
    return E


def fci_hamiltonian(h: np.ndarray, V: np.ndarray, n_a: int, n_b: int, fs: FockSpace | None = None):
    """Sparse FCI Hamiltonian in the (n_a, n_b) sector and the basis states."""
    n = h.shape[0]
    fs = fs or FockSpace(n)
    idx = sector_basis(fs, n_a, n_b)
    E = excitation_ops(fs, idx)
    dim = len(idx)
    H = sp.csr_matrix((dim, dim))
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                H = H + h[p, q] * E[p][q]
    for p in range(n):
        for q in range(n):
            F = sp.csr_matrix((dim, dim))
            for r in range(n):
                for s in range(n):
                    if V[p, q, r, s] != 0.0:
                        F = F + V[p, q, r, s] * E[r][s]
            H = H + 0.5 * (E[p][q] @ F)
    for p in range(n):
        for s in range(n):
            c = sum(V[p, q, q, s] for q in range(n))
            if c != 0.0:
                H = H - 0.5 * c * E[p][s]
    return H.tocsr(), idx


def fci_energy(h, V, n_a, n_b, dense: bool = False):
    H, _ = fci_hamiltonian(h, V, n_a, n_b)
    if dense or H.shape[0] <= 64:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    w = spla.eigsh(H, k=1, which="SA", tol=1e-14, maxiter=100000)[0]
    return float(w[0])


def fci_rdm1(h, V, n_a, n_b):
    """Ground state of the (n_a, n_b) sector by dense diagonalisation and its
    spin-summed one-particle density matrix gamma_pq = <Psi|E_pq|Psi>.
    Returns (E0, gamma, gap to the next eigenvalue); gamma is defined only
    for a non-degenerate ground state (the gap says whether it is)."""
    n = h.shape[0]
    fs = FockSpace(n)
    H, idx = fci_hamiltonian(h, V, n_a, n_b, fs)
    w, U = np.linalg.eigh(H.toarray())
    c = U[:, 0]
    E = excitation_ops(fs, idx)
    gamma = np.array([[c @ (E[p][q] @ c) for q in range(n)] for p in range(n)])
    gap = float(w[1] - w[0]) if len(w) > 1 else np.inf
    return float(w[0]), gamma, gap

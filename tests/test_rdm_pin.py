"""The derivative of the ground-state energy with respect to the one-electron
integrals, taken through the operator build, equals the FCI one-particle
density matrix: dE/dh_pq = <Psi| sum_s a+_ps a_qs |Psi> = gamma_pq.

The operator pairs are linear in (h, V) for fixed block bases, so the
derivative through the build is psi^T H_eff(E_pq, V = 0) psi with psi the
ground state of H_eff(h, V) and E_pq the unit matrix at (p, q) (Hellmann-
Feynman).  At full bond dimension (L <= 6) the two-site space is the whole
FCI sector, so the two sides must agree to rounding.  Checked for the
oracle's own pair builder and for the library's chain (its host-side build,
applied by the oracle's matvec).  The 1-RDM itself is pinned by its trace,
its symmetry, the closed-shell V = 0 closed form and central differences of
the FCI energy."""
import numpy as np
import pytest

from oracle.fci import fci_energy, fci_rdm1
from oracle.heff import heff_apply, heff_dense
from oracle.physical import physical_problem
from synth.integrals import integrals

CASES = [(4, 2, 2, 31), (5, 3, 2, 32), (6, 3, 3, 33)]


def _unit(L, p, q):
    e = np.zeros((L, L))
    e[p, q] = 1.0
    return e


def test_rdm1_pins():
    L, na, nb = 5, 2, 2
    h, V = integrals(L, 41)
    E0, g, gap = fci_rdm1(h, V, na, nb)
    assert gap > 1e-3
    assert abs(np.trace(g) - (na + nb)) < 1e-12
    assert np.abs(g - g.T).max() < 1e-12
    # central differences of the FCI energy along symmetric perturbations
    # S = E_pq + E_qp (p != q) or E_pp: dE/d eps = gamma_pq + gamma_qp, or gamma_pp
    eps = 1e-5
    for p, q in [(0, 0), (1, 3), (4, 2)]:
        S = _unit(L, p, q) + (_unit(L, q, p) if p != q else 0.0)
        ep = fci_energy(h + eps * S, V, na, nb, dense=True)
        em = fci_energy(h - eps * S, V, na, nb, dense=True)
        fd = (ep - em) / (2 * eps) / (2.0 if p != q else 1.0)
        assert abs(fd - g[p, q]) < 1e-7
    # V = 0, closed shell: gamma = 2 C_occ C_occ^T from the orbitals of h
    hs = 0.5 * (h + h.T)
    _, g0, gap0 = fci_rdm1(hs, np.zeros_like(V), na, na)
    w, C = np.linalg.eigh(hs)
    assert gap0 > 1e-6 and w[na] - w[na - 1] > 1e-6
    assert np.abs(g0 - 2.0 * C[:, :na] @ C[:, :na].T).max() < 1e-12


def _ground(prob):
    H = heff_dense(prob)
    w, U = np.linalg.eigh(H)
    return w, U[:, 0]


@pytest.mark.parametrize("L,na,nb,seed", CASES)
def test_energy_gradient_through_oracle_build_is_rdm1(L, na, nb, seed):
    h, V = integrals(L, seed)
    E0, g, gap = fci_rdm1(h, V, na, nb)
    assert gap > 1e-4
    m = L // 2 - 1
    prob = physical_problem(h, V, m, na, nb)
    w, psi = _ground(prob)
    assert abs(w[0] - E0) < 1e-10
    zero = np.zeros_like(V)
    for p in range(L):
        for q in range(L):
            d = psi @ heff_apply(physical_problem(_unit(L, p, q), zero, m, na, nb), psi)
            assert abs(d - g[p, q]) < 1e-10, (p, q, d, g[p, q])


@pytest.mark.parametrize("L,na,nb,seed", CASES)
def test_energy_gradient_through_library_build_is_rdm1(L, na, nb, seed):
    from paper_2407_07411_amd.chain import Chain
    h, V = integrals(L, seed)
    E0, g, gap = fci_rdm1(h, V, na, nb)
    prob = Chain(None, h, V, na + nb, na - nb, D=4 ** L, seed=3).export(0)
    w, psi = _ground(prob)
    assert abs(w[0] - E0) < 1e-10
    zero = np.zeros_like(V)
    for p in range(L):
        for q in range(L):
            pq = Chain(None, _unit(L, p, q), zero, na + nb, na - nb, D=4 ** L, seed=3).export(0)
            d = psi @ heff_apply(pq, psi)
            assert abs(d - g[p, q]) < 1e-10, (p, q, d, g[p, q])

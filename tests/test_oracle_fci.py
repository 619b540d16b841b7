"""Pins of the FCI oracle against closed forms and invariants.

The paper's variational energy (Eq. 2) at unlimited bond dimension is the
FCI energy; these checks fix the FCI oracle without trusting its own
arithmetic: dimension counts, symmetry, the non-interacting limit, the
Hubbard dimer, the Hartree-Fock diagonal element and orbital-permutation
invariance.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.fci import fci_energy, fci_hamiltonian
from oracle.fock import FockSpace
from synth.integrals import hubbard_dimer, integrals


@pytest.fixture(scope="module")
def l8():
    h, V = integrals(8, 1001)
    H, idx = fci_hamiltonian(h, V, 4, 4)
    return h, V, H, idx


def test_l8_dimension(l8):
    _, _, H, idx = l8
    # C(8,4)^2 determinants for 4 alpha + 4 beta electrons in 8 orbitals
    assert H.shape == (4900, 4900) and len(idx) == 4900


def test_l8_symmetric(l8):
    _, _, H, _ = l8
    assert abs(H - H.T).max() <= 1e-13 * abs(H).max()


def test_integral_symmetries():
    h, V = integrals(6, 5)
    assert np.array_equal(h, h.T)
    for perm in ["jikl", "ijlk", "klij", "jilk", "lkji", "lkij", "klji"]:
        assert np.allclose(V, np.einsum("ijkl->" + perm, V), atol=0, rtol=0) or \
            np.abs(V - np.einsum("ijkl->" + perm, V)).max() < 1e-15
    # positive semidefinite as a pair-space supermatrix
    M = V.reshape(36, 36)
    assert np.linalg.eigvalsh(M).min() > -1e-12


def test_noninteracting_closed_form():
    h, _ = integrals(6, 11)
    V = np.zeros((6,) * 4)
    eps = np.linalg.eigvalsh(h)
    for (na, nb) in [(3, 3), (2, 1), (4, 2), (0, 3)]:
        e = fci_energy(h, V, na, nb, dense=True)
        assert abs(e - (eps[:na].sum() + eps[:nb].sum())) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 0.0), (1.0, 4.0), (0.5, 8.0), (2.0, 1.3)])
def test_hubbard_dimer(t, U):
    h, V = hubbard_dimer(t, U)
    e = fci_energy(h, V, 1, 1, dense=True)
    assert abs(e - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-13


def test_hartree_fock_diagonal(l8):
    h, V, H, idx = l8
    # determinant with orbitals 0..3 doubly occupied: modes 0..7 set
    x_hf = (1 << 8) - 1
    k = int(np.nonzero(idx == x_hf)[0][0])
    occ = range(4)
    ref = 2 * sum(h[i, i] for i in occ) + sum(
        2 * V[i, i, j, j] - V[i, j, j, i] for i in occ for j in occ)
    assert abs(H[k, k] - ref) < 1e-12


def test_orbital_permutation_invariance():
    h, V = integrals(6, 3)
    perm = np.array([3, 0, 5, 1, 4, 2])
    hp = h[np.ix_(perm, perm)]
    Vp = V[np.ix_(perm, perm, perm, perm)]
    e1 = fci_energy(h, V, 3, 2, dense=True)
    e2 = fci_energy(hp, Vp, 3, 2, dense=True)
    assert abs(e1 - e2) < 1e-11


def test_lanczos_matches_dense():
    h, V = integrals(6, 13)
    H, _ = fci_hamiltonian(h, V, 3, 3)
    dense = np.linalg.eigvalsh(H.toarray())[0]
    lan = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(dense - lan) < 1e-10


def test_fock_operators_anticommute():
    fs = FockSpace(2)
    I = np.eye(fs.dim)
    for m in range(4):
        for n in range(4):
            am, an = fs._a[m].toarray(), fs._a[n].toarray()
            assert np.array_equal(am @ an.T + an.T @ am, I if m == n else 0 * I)
            assert np.array_equal(am @ an + an @ am, 0 * I)

"""Pins of the operator-sum matvec oracle.

* brute force: the column-by-column matvec equals an independently
  assembled dense sum of Kronecker products over the full enlarged spaces,
  restricted to the wavefunction's blocks;
* physics: with operator pairs of the real Hamiltonian, the operator sum is
  P^T H_FCI P, and at the L=8 centre bond (full Fock blocks) its ground
  state is the FCI energy;
* invariants: Hermiticity, linearity, the diagonal, and the reduction of a
  single dq = 0 term to A Psi B^T.
"""
import numpy as np
import pytest
import torch

from oracle.davidson import davidson
from oracle.fci import fci_energy, fci_hamiltonian
from oracle.heff import count_bytes, count_flops, heff_apply, heff_dense, heff_diag, layout_of
from oracle.physical import embedding, physical_problem
from synth.integrals import integrals
from synth.problem import Problem, Term
from tests.conftest import tiny_problem, with_one_sided_hc


def kron_dense(prob):
    """Dense H_eff from full-space Kronecker products (independent path)."""
    Lq, Ld, Rq, Rd = np.asarray(prob.Lq), np.asarray(prob.Ld), np.asarray(prob.Rq), np.asarray(prob.Rd)
    lo = np.concatenate([[0], np.cumsum(Ld)])
    ro = np.concatenate([[0], np.cumsum(Rd)])
    nl, nr = lo[-1], ro[-1]
    lp, rp = prob.left_pool.numpy(), prob.right_pool.numpy()
    lid = {tuple(q): i for i, q in enumerate(Lq.tolist())}
    rid = {tuple(q): i for i, q in enumerate(Rq.tolist())}
    Z = np.diag(np.concatenate([np.full(Ld[a], (-1.0) ** Lq[a][0]) for a in range(len(Ld))]))
    H = np.zeros((nl * nr, nl * nr))
    for t in prob.terms:
        A = np.eye(nl)
        B = np.eye(nr)
        if t.one_sided != 2:
            A = np.zeros((nl, nl))
            for a, q in enumerate(Lq.tolist()):
                b = lid.get((q[0] + t.dq[0], q[1] + t.dq[1]))
                if t.left_off[a] >= 0:
                    blk = lp[t.left_off[a]:t.left_off[a] + Ld[b] * Ld[a]].reshape(Ld[b], Ld[a])
                    A[lo[b]:lo[b + 1], lo[a]:lo[a + 1]] = blk
        if t.one_sided != 1:
            B = np.zeros((nr, nr))
            for c, r in enumerate(Rq.tolist()):
                e = rid.get((r[0] - t.dq[0], r[1] - t.dq[1]))
                if t.right_off[c] >= 0:
                    blk = rp[t.right_off[c]:t.right_off[c] + Rd[e] * Rd[c]].reshape(Rd[e], Rd[c])
                    B[ro[e]:ro[e + 1], ro[c]:ro[c + 1]] = blk
        Zp = Z if t.odd else np.eye(nl)
        H += t.coeff * np.kron(A @ Zp, B)
        if t.hc:
            H += (-t.coeff if t.odd else t.coeff) * np.kron(A.T @ Zp, B.T)
    # restrict to the wavefunction's blocks
    lay = layout_of(prob)
    sel = []
    for a in lay.partner:
        c = lay.partner[a]
        for i in range(Ld[a]):
            for j in range(Rd[c]):
                sel.append((lo[a] + i) * nr + ro[c] + j)
    sel = np.array(sel)
    return H[np.ix_(sel, sel)]


@pytest.mark.parametrize("one_sided_hc", [False, True])
@pytest.mark.parametrize("seed,D,two_sz", [(1, 4, 0), (2, 6, 0), (3, 5, 2)])
def test_matvec_equals_kron_assembly(seed, D, two_sz, one_sided_hc):
    prob = tiny_problem(seed=seed, D=D, two_sz=two_sz, pairs=2)
    if one_sided_hc:
        prob = with_one_sided_hc(prob, seed=seed)
    H1 = heff_dense(prob)
    H2 = kron_dense(prob)
    assert np.abs(H1 - H2).max() <= 1e-13 * max(1.0, np.abs(H2).max())


def test_hermitian_and_linear():
    prob = tiny_problem(seed=4, D=10, pairs=3)
    n = layout_of(prob).total
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Hx, Hy = heff_apply(prob, x), heff_apply(prob, y)
    norm = np.linalg.norm(heff_dense(prob), 2)
    assert abs(x @ Hy - Hx @ y) <= 1e-13 * norm * np.linalg.norm(x) * np.linalg.norm(y)
    assert np.allclose(heff_apply(prob, 2.5 * x - y), 2.5 * Hx - Hy, rtol=0, atol=1e-12)
    # linear in the operator pools (each two-sided term is bilinear in (A, B))
    lp2 = prob.left_pool * 3.0
    y1 = heff_apply(prob, x)
    y3 = heff_apply(prob, x, left_pool=lp2)
    only_right = sum(1 for t in prob.terms if t.one_sided == 2)
    assert only_right == 1
    yr = heff_apply(prob, x, terms=[t for t in prob.terms if t.one_sided == 2])
    assert np.allclose(y3 - yr, 3.0 * (y1 - yr), rtol=0, atol=1e-12)


@pytest.mark.parametrize("one_sided_hc", [False, True])
def test_diag_matches_dense(one_sided_hc):
    prob = tiny_problem(seed=5, D=8, pairs=3)
    if one_sided_hc:
        prob = with_one_sided_hc(prob, seed=5)
    assert np.abs(heff_diag(prob) - np.diag(heff_dense(prob))).max() < 1e-13


def test_single_term_is_A_psi_Bt():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    B = rng.standard_normal((4, 4))
    P = rng.standard_normal((3, 4))
    t = Term(dq=(0, 0), odd=0, hc=0, one_sided=0, coeff=0.7,
             left_off=np.array([0]), right_off=np.array([0]))
    prob = Problem(np.array([[1, 1]], dtype=np.int32), np.array([3]), np.array([[2, 0]], dtype=np.int32),
                   np.array([4]), np.array([3, 1], dtype=np.int32), [t],
                   torch.from_numpy(A.ravel().copy()), torch.from_numpy(B.ravel().copy()),
                   torch.from_numpy(P.ravel().copy()))
    y = heff_apply(prob)
    assert np.allclose(y, (0.7 * A @ P @ B.T).ravel(), rtol=0, atol=1e-14)


def _random_isometries(fs, keep, rng):
    iso = {}
    for q in sorted({tuple(q) for q in fs.qn.tolist()}):
        n = len(fs.sector(*q))
        k = min(n, keep)
        M = rng.standard_normal((n, k))
        iso[q] = np.linalg.qr(M)[0]
    return iso


@pytest.mark.parametrize("L,m,na,nb,keep", [(4, 2, 2, 2, 99), (5, 2, 3, 2, 99), (5, 3, 2, 2, 2), (6, 3, 3, 3, 3)])
def test_physical_pairs_are_projected_fci(L, m, na, nb, keep):
    from oracle.fock import FockSpace
    h, V = integrals(L, 21 + L)
    rng = np.random.default_rng(L * 10 + m)
    isoL = _random_isometries(FockSpace(m), keep, rng)
    isoR = _random_isometries(FockSpace(L - m), keep, rng)
    prob = physical_problem(h, V, m, na, nb, isoL, isoR)
    H, idx = fci_hamiltonian(h, V, na, nb)
    P = embedding(prob, idx)
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-13        
    He = heff_dense(prob)
    Hp = P.T @ (H @ P)
    assert np.abs(He - Hp).max() < 1e-12 * max(1.0, np.abs(Hp).max())
    assert np.abs(He - He.T).max() < 1e-12                              
    e_fci = fci_energy(h, V, na, nb, dense=True)
    assert np.linalg.eigvalsh(He)[0] >= e_fci - 1e-10                   


def test_l8_centre_recovers_fci():
    """L=8 centre two-site step: blocks of 4 orbitals hold every Fock
    state (64 = D states per 3-orbital block, times the 4 site states), so
    the two-site space is the full 4900-dim FCI space."""
    h, V = integrals(8, 1001)
    prob = physical_problem(h, V, 4, 4, 4)
    lay = layout_of(prob)
    assert lay.total == 4900
    e_fci = fci_energy(h, V, 4, 4)
    # the lowest Sz=0 state of these integrals is a triplet component (odd
    # under alpha<->beta exchange), so a closed-shell start vector cannot
    # reach it; start from a seeded random vector instead
    x0 = np.random.default_rng(8).standard_normal(lay.total)
    res = davidson(lambda v: heff_apply(prob, v), heff_diag(prob), x0=x0, tol=1e-8)
    assert res["converged"]
    assert abs(res["energy"] - e_fci) < 1e-9


def test_l8_ground_state_is_triplet():
    h, V = integrals(8, 1001)
    assert abs(fci_energy(h, V, 5, 3) - fci_energy(h, V, 4, 4)) < 1e-9


def test_flop_count_by_hand():
    # one two-sided term, dq=0, one block 3x4 with A 3x3, B 4x4:
    # left-first 2*3*3*4 + 2*3*4*4 = 72 + 96 = 168, right-first 96 + 72 = 168
    rng = np.random.default_rng(3)
    t = Term(dq=(0, 0), odd=0, hc=1, one_sided=0, coeff=1.0,
             left_off=np.array([0]), right_off=np.array([0]))
    prob = Problem(np.array([[1, 1]], dtype=np.int32), np.array([3]), np.array([[2, 0]], dtype=np.int32),
                   np.array([4]), np.array([3, 1], dtype=np.int32), [t],
                   torch.from_numpy(rng.standard_normal(9)), torch.from_numpy(rng.standard_normal(16)),
                   torch.zeros(12, dtype=torch.float64))
    assert count_flops(prob) == 2 * 168
    # bytes: A (9) and B (16) read once (the hc partner reuses them), psi
    # read and y written (12 each)
    assert count_bytes(prob) == 8 * (9 + 16 + 2 * 12)


def _rect_problem(one_sided=0, hc=0):
    """Two left sectors (1,1) d=3 and (2,0) d=2, two right sectors (2,0) d=4
    and (1,1) d=5, total Q = (3,1): psi blocks 3x4 (a0, c0) and 2x5 (a1, c1)."""
    rng = np.random.default_rng(5)
    Lq = np.array([[1, 1], [2, 0]], dtype=np.int32)
    Rq = np.array([[2, 0], [1, 1]], dtype=np.int32)
    Ld, Rd = np.array([3, 2]), np.array([4, 5])
    if one_sided == 0:
        # dq = (1,-1), odd: O^L[a1, a0] is 2x3, O^R[c1, c0] is 5x4
        t = Term(dq=(1, -1), odd=1, hc=hc, one_sided=0, coeff=0.5,
                 left_off=np.array([0, -1]), right_off=np.array([0, -1]))
        lp, rp = rng.standard_normal(6), rng.standard_normal(20)
    elif one_sided == 1:
        t = Term(dq=(0, 0), odd=0, hc=hc, one_sided=1, coeff=0.5,
                 left_off=np.array([0, 9]), right_off=None)
        lp, rp = rng.standard_normal(13), rng.standard_normal(1)
    else:
        t = Term(dq=(0, 0), odd=0, hc=hc, one_sided=2, coeff=0.5,
                 left_off=None, right_off=np.array([0, 16]))
        lp, rp = rng.standard_normal(1), rng.standard_normal(41)
    return Problem(Lq, Ld, Rq, Rd, np.array([3, 1], dtype=np.int32), [t], torch.from_numpy(lp),
                   torch.from_numpy(rp), torch.from_numpy(rng.standard_normal(22)))


@pytest.mark.parametrize("hc", [0, 1])
def test_flop_count_rectangular_shift_by_hand(hc):
    # item (a0,c0) 3x4 -> (a1,c1) 2x5 with A 2x3, B 5x4:
    #   left-first  A Psi: 2*2*3*4 = 48, then (2x4) B^T: 2*2*4*5 = 80 -> 128
    #   right-first Psi B^T: 2*3*4*5 = 120, then A (3x5): 2*2*3*5 = 60 -> 180
    # partner (a1,c1) 2x5 -> (a0,c0) 3x4 with A^T 3x2, B^T 4x5:
    #   left-first  A^T Psi: 2*3*2*5 = 60, then (3x5) B: 2*3*5*4 = 120 -> 180
    #   right-first Psi B: 2*2*5*4 = 80, then A^T (2x4): 2*3*2*4 = 48 -> 128
    prob = _rect_problem(0, hc)
    assert count_flops(prob) == 128 * (1 + hc)
    # both items read the same two stored blocks: 6 + 20 doubles, psi 22
    assert count_bytes(prob) == 8 * (6 + 20 + 2 * 22)
    # the item list behind it: the dense operator has exactly these blocks
    H = heff_dense(prob)
    assert np.count_nonzero(H[12:, :12]) == 10 * 12
    assert np.count_nonzero(H[:12, 12:]) == (12 * 10 if hc else 0)


@pytest.mark.parametrize("one_sided", [1, 2])
@pytest.mark.parametrize("hc", [0, 1])
def test_flop_count_one_sided_by_hand(one_sided, hc):
    # left only: A_q Psi_q per block, 2*3*3*4 = 72 and 2*2*2*5 = 40;
    # right only: Psi_q B_q^T, 2*3*4*4 = 96 and 2*2*5*5 = 100; hc doubles
    prob = _rect_problem(one_sided, hc)
    per = 72 + 40 if one_sided == 1 else 96 + 100
    assert count_flops(prob) == per * (1 + hc)
    blocks = 9 + 4 if one_sided == 1 else 16 + 25
    assert count_bytes(prob) == 8 * (blocks + 2 * 22)


@pytest.mark.parametrize("seed,D,two_sz", [(4, 6, 0), (5, 5, 2)])
def test_sampled_entries_equal_kron_assembly(seed, D, two_sz):
    """heff_entries (used to sample whole-size problems) against the
    independent Kronecker assembly, on every block and a ragged sample."""
    from oracle.heff import heff_entries
    prob = tiny_problem(seed=seed, D=D, two_sz=two_sz, pairs=2)
    lay = layout_of(prob)
    x = prob.psi.numpy()
    y = kron_dense(prob) @ x
    for b in lay.partner:
        e = lay.partner[b]
        nr, nc = int(lay.Ld[b]), int(lay.Rd[e])
        rows = list(range(nr))[::2] or [0]
        cols = list(range(nc))[::-1]
        val, mag = heff_entries(prob, b, rows, cols)
        ref = lay.block(y, b)[np.ix_(rows, cols)]
        assert np.abs(val - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
        assert np.all(mag >= np.abs(val) - 1e-15)


@pytest.mark.parametrize("one_sided_hc", [False, True])
def test_sampled_blocks_equal_kron_assembly(one_sided_hc):
    """heff_entries_blocks (every output block of a whole-size problem in one
    pass) against the Kronecker assembly and against heff_entries."""
    from oracle.heff import heff_entries, heff_entries_blocks
    prob = tiny_problem(seed=6, D=7, two_sz=0, pairs=3)
    if one_sided_hc:
        prob = with_one_sided_hc(prob, seed=6)
    lay = layout_of(prob)
    y = kron_dense(prob) @ prob.psi.numpy()
    samples = {}
    for b in lay.partner:
        nr, nc = int(lay.Ld[b]), int(lay.Rd[lay.partner[b]])
        samples[b] = (sorted({0, nr - 1}), sorted({0, nc // 2, nc - 1}))
    got = heff_entries_blocks(prob, samples)
    assert set(got) == set(samples)
    for b, (rows, cols) in samples.items():
        val, mag = got[b]
        ref = lay.block(y, b)[np.ix_(rows, cols)]
        assert np.abs(val - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
        v1, m1 = heff_entries(prob, b, rows, cols)
        assert np.allclose(val, v1, rtol=0, atol=1e-13 * max(1.0, np.abs(v1).max()))
        assert np.allclose(mag, m1, rtol=1e-13, atol=0)

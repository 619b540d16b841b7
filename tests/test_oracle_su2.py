"""Pins of the SU(2) spin-adapted oracle (oracle/su2.py), on the CPU.

* Clebsch-Gordan coefficients: orthonormality of the coupled basis, the
  Condon-Shortley values of two spin-1/2 and two spin-1 particles, stretched
  and trivial couplings, and the Wigner-Eckart decomposition of the textbook
  spin operators S_z, S_+ (matrix elements m and sqrt(j(j+1) - m(m+1)))
  into one reduced element per j.
* The recoupling weight is independent of M (Wigner-Eckart theorem).
* The reduced matvec, expanded into the U(1) x U(1) basis through the same
  coefficients, equals oracle.heff (itself pinned against Kronecker assembly
  and FCI) applied to the expanded problem, at every M, on problems with
  half-integer spins, fermion-odd terms and hermitian-conjugate partners.
* The diagonal and the FLOP count follow their definitions.
* The library's host weight (6j closed form) equals the oracle's CG-sum
  definition for every spin combination up to 2j = 8, 2k = 4."""
import itertools
from math import sqrt

import numpy as np
import pytest

from oracle.heff import heff_apply
from oracle.su2 import (_tri, cg, count_flops_su2, expand_to_u1, heff_apply_su2, heff_dense_su2,
                        heff_diag_su2, layout_su2, weight)
from synth.su2 import tiny_su2


def test_cg_orthonormal():
    for tj1, tj2 in itertools.product(range(0, 7), range(0, 7)):
        states = [(tm1, tm2) for tm1 in range(-tj1, tj1 + 1, 2) for tm2 in range(-tj2, tj2 + 1, 2)]
        coupled = [(tJ, tM) for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2) for tM in range(-tJ, tJ + 1, 2)]
        U = np.array([[cg(tj1, a, tj2, b, tJ, tM) for (a, b) in states] for (tJ, tM) in coupled])
        assert U.shape[0] == U.shape[1]
        assert np.abs(U @ U.T - np.eye(len(states))).max() < 1e-13


def test_cg_values():
    r2, r3 = sqrt(0.5), sqrt(1.0 / 3.0)
    assert abs(cg(1, 1, 1, -1, 2, 0) - r2) < 1e-15
    assert abs(cg(1, -1, 1, 1, 2, 0) - r2) < 1e-15
    assert abs(cg(1, 1, 1, -1, 0, 0) - r2) < 1e-15
    assert abs(cg(1, -1, 1, 1, 0, 0) + r2) < 1e-15
    for tm, sgn in ((2, 1.0), (0, -1.0), (-2, 1.0)):
        assert abs(cg(2, tm, 2, -tm, 0, 0) - sgn * r3) < 1e-15
    for tj1, tj2 in itertools.product(range(0, 9), range(0, 9)):
        assert abs(cg(tj1, tj1, tj2, tj2, tj1 + tj2, tj1 + tj2) - 1.0) < 1e-14
    for tj in range(0, 9):
        for tm in range(-tj, tj + 1, 2):
            assert abs(cg(tj, tm, 0, 0, tj, tm) - 1.0) < 1e-15
    assert cg(2, 0, 2, 0, 2, 0) == 0.0
    assert cg(1, 1, 1, 1, 0, 2) == 0.0


def test_cg_reproduce_spin_operators():
    """<j m'|S_q|j m> = <j m; 1 q|j m'> <j||S||j> with S_0 = S_z and
    S_{+1} = -S_+/sqrt(2): one reduced element per j, equal from both."""
    for tj in range(1, 9):
        j = tj / 2
        red = set()
        for tm in range(-tj, tj + 1, 2):
            m = tm / 2
            c0 = cg(tj, tm, 2, 0, tj, tm)
            if abs(c0) > 1e-12:
                red.add(round(m / c0, 12))
            if tm + 2 <= tj:
                splus = sqrt(j * (j + 1) - m * (m + 1))
                red.add(round(-splus / sqrt(2.0) / cg(tj, tm, 2, 2, tj, tm + 2), 12))
        assert len(red) == 1, (tj, red)
        assert abs(next(iter(red)) - sqrt(j * (j + 1))) < 1e-12


def test_weight_independent_of_m():
    for tja, tjc, tja2, tjc2, tk, tS in itertools.product(range(5), range(5), range(5), range(5), range(3),
                                                         range(5)):
        if not (_tri(tja, tjc, tS) and _tri(tja2, tjc2, tS)):
            continue
        ws = [weight(tja, tjc, tja2, tjc2, tk, tS, tM) for tM in range(-tS, tS + 1, 2)]
        assert max(ws) - min(ws) < 1e-13


CASES = [dict(seed=1, N=6, two_s=0), dict(seed=2, N=5, two_s=1), dict(seed=3, N=6, two_s=2),
         dict(seed=4, N=5, two_s=3), dict(seed=5, N=4, two_s=4, n_hi=3, tj_max=2),
         dict(seed=6, N=7, two_s=1, n_hi=5, tj_max=3, dmax=2)]


@pytest.mark.parametrize("kw", CASES)
def test_reduced_matvec_equals_u1_expansion(kw):
    prob = tiny_su2(**kw)
    y = heff_apply_su2(prob)
    assert np.linalg.norm(y) > 0.1
    groups = {t.group for t in prob.terms}
    assert {"CS", "SA", "AP1", "BQ1", "HL", "HR"} <= groups
    tS = int(prob.Q[1])
    for tM in range(tS, -tS - 1, -2):
        up, expand = expand_to_u1(prob, tM)
        yu = heff_apply(up)
        assert np.abs(yu - expand(y)).max() < 1e-13 * max(1.0, np.abs(yu).max())
        # the expansion is an isometry
        assert abs(np.linalg.norm(up.psi) - 1.0) < 1e-13


def test_u1_expansion_catches_a_wrong_phase():
    """A planted mistake (the sign of one fermion-odd term's weight) breaks
    the equality: the pin sees conventions, not just norms."""
    import dataclasses
    prob = tiny_su2(seed=2, N=5, two_s=1)
    odd = [i for i, t in enumerate(prob.terms) if t.odd]
    bad = list(prob.terms)
    bad[odd[0]] = dataclasses.replace(bad[odd[0]], coeff=-bad[odd[0]].coeff)
    y_bad = heff_apply_su2(dataclasses.replace(prob, terms=bad))
    up, expand = expand_to_u1(prob)
    assert np.abs(heff_apply(up) - expand(y_bad)).max() > 1e-3


def test_dense_symmetric_diag_and_flops():
    prob = tiny_su2(seed=3, N=6, two_s=2)
    H = heff_dense_su2(prob)
    assert np.abs(H - H.T).max() < 1e-13
    assert np.abs(np.diag(H) - heff_diag_su2(prob)).max() < 1e-13
    # FLOPs by hand for a single one-sided left term: 2 d_a^2 d_c per block
    import dataclasses
    one = [t for t in prob.terms if t.group == "HL"]
    p1 = dataclasses.replace(prob, terms=one)
    lay = layout_su2(p1)
    hand = sum(2 * int(lay.Ld[a]) ** 2 * int(lay.Rd[c]) for (a, c) in lay.blocks)
    assert count_flops_su2(p1) == hand


def test_library_weight_equals_oracle():
    """dmrg_su2_weight (the library's 6j closed form, a host call) against
    the oracle's definition as a Clebsch-Gordan sum."""
    from paper_2407_07411_amd.heff import su2_weight
    n = 0
    for tja, tjc, tja2, tjc2, tk, tS in itertools.product(range(9), range(9), range(9), range(9), range(5),
                                                         range(9)):
        if not (_tri(tja, tjc, tS) and _tri(tja2, tjc2, tS) and _tri(tja, tk, tja2) and _tri(tjc, tk, tjc2)):
            assert su2_weight(tja, tjc, tja2, tjc2, tk, tS) == 0.0 or not _tri(tja, tjc, tS)
            continue
        w = weight(tja, tjc, tja2, tjc2, tk, tS)
        assert abs(su2_weight(tja, tjc, tja2, tjc2, tk, tS) - w) < 1e-13, (tja, tjc, tja2, tjc2, tk, tS)
        n += 1
    assert n > 2000


@pytest.mark.parametrize("kw", [CASES[0], CASES[3], dict(seed=11, n_lo=2, n_hi=7, tj_max=5, dmax=12, N=9,
                                                           two_s=1, pairs=3)])
def test_sampled_entries_equal_full_matvec(kw):
    """heff_entries_blocks_su2 (items formed per sampled output block, rows
    gathered from the pools) reproduces every block of heff_apply_su2."""
    from oracle.su2 import heff_entries_blocks_su2
    prob = tiny_su2(**kw)
    lay = layout_su2(prob)
    y = heff_apply_su2(prob)
    samples = {b: (list(range(int(lay.Ld[b[0]]))), list(range(int(lay.Rd[b[1]])))) for b in lay.blocks}
    got = heff_entries_blocks_su2(prob, samples)
    for b in lay.blocks:
        val, mag = got[b]
        assert np.abs(lay.block(y, *b) - val).max() <= 1e-13 * max(1.0, mag.max())
        assert np.all(mag >= np.abs(val) - 1e-13)

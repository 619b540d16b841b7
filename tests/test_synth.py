"""Generator checks: determinism, sector tables, term counts, pool sizes."""
import numpy as np

from synth.problem import WORKLOADS, group_counts, psi_layout
from synth.sectors import bond_sectors, block_sectors
from tests.conftest import tiny_problem


def test_deterministic_sha():
    a = tiny_problem(seed=3, D=6).sha256()
    b = tiny_problem(seed=3, D=6).sha256()
    c = tiny_problem(seed=4, D=6).sha256()
    assert a == b and a != c


def test_block_sectors_sum_to_D():
    for (L, N, s2, D) in [(24, 24, 0, 1024), (58, 63, 1, 4096), (76, 113, 3, 8192)]:
        lb, rb = block_sectors(L, (N + s2) // 2, (N - s2) // 2, D)
        assert sum(d for _, d in lb) == D and sum(d for _, d in rb) == D


def test_sector_tables_shapes():
    # enlarged sector counts, largest sector and wavefunction size
    expect = {"l24_d1024": (94, 209, 402285), "cas63_58_d4096": (120, 834, 6946846),
              "cas113_76_d8192": (124, 1667, 27836254)}
    for name, w in WORKLOADS.items():
        Lq, Ld, Rq, Rd, Q = bond_sectors(w["L"], w["n_elec"], w["two_sz"], w["D"])
        assert Ld.sum() == 4 * w["D"] and Rd.sum() == 4 * w["D"]
        _, total = psi_layout(Lq, Ld, Rq, Rd, Q)
        assert (len(Ld), int(Ld.max()), total) == expect[name]


def test_term_counts():
    # stored pairs and terms (hermitian-conjugate partners counted)
    for k, pairs, terms in [(12, 626, 1226), (29, 3482, 6904), (38, 5930, 11782)]:
        c = group_counts(k, k)
        assert sum(c.values()) == pairs
        hc = {"CS_a", "CS_b", "SA_a", "SA_b", "AP_aa", "AP_bb", "AP_ab", "BQ_off", "BQ_flip"}
        assert sum(n * (2 if g in hc else 1) for g, n in c.items()) == terms


def test_psi_unit_norm_and_blocks_symmetric():
    p = tiny_problem(seed=5, D=10)
    assert abs(float(p.psi.norm()) - 1.0) < 1e-14
    lp = p.left_pool.numpy()
    for t in p.terms:
        if t.group in ("HL", "BQ_diag"):
            for a, off in enumerate(t.left_off):
                if off >= 0:
                    d = int(p.Ld[a])
                    blk = lp[off:off + d * d].reshape(d, d)
                    assert np.array_equal(blk, blk.T)


def test_su2_bond_sectors():
    """Multiplet tables of the SU(2) workloads: electron parity (2j = N mod
    2); most sectors of each enlarged block pair with one on the other side
    into the total (N, S) (the rest carry no wavefunction block, as in a
    real enlarged basis); and the enlarged block holds 4x the states of the
    block (one site: j x {0, 1/2, 0} with the 1/2 splitting j into j -+ 1/2)."""
    from synth.su2 import WORKLOADS_SU2, _psi_blocks, bond_sectors_su2
    for name, w in WORKLOADS_SU2.items():
        Lq, Ld, Rq, Rd, Q = bond_sectors_su2(w["L"], w["n_elec"], w["two_s"], w["D"])
        for q in (Lq, Rq):
            assert all(int(N) % 2 == int(tj) % 2 and tj >= 0 for N, tj in q.tolist())
        blocks = _psi_blocks(Lq, Rq, Q)
        assert len({a for a, _ in blocks}) >= 0.75 * len(Lq)
        assert len({c for _, c in blocks}) >= 0.75 * len(Rq)
        assert int(Ld.sum()) > w["D"] and int(Rd.sum()) > w["D"]
        # total states of the enlarged block = 4 x the block's states
        for q, d in ((Lq, Ld), (Rq, Rd)):
            states = sum(int(n) * (int(tj) + 1) for (_, tj), n in zip(q.tolist(), d.tolist()))
            assert states % 4 == 0


def test_su2_problem_blocks_obey_selection_rules():
    from synth.su2 import tiny_su2
    p = tiny_su2(seed=3, N=6, two_s=2)
    for t in p.terms:
        for tab, q, dn in ((t.left_blocks, p.Lq, t.dn), (t.right_blocks, p.Rq, -t.dn)):
            if tab is None:
                continue
            for o, i, _ in np.asarray(tab).tolist():
                assert int(q[o][0]) - int(q[i][0]) == dn
                tj, tk, tj2 = int(q[i][1]), t.two_k, int(q[o][1])
                assert abs(tj - tk) <= tj2 <= tj + tk and (tj + tk + tj2) % 2 == 0

"""The allocation-free truncating SVD (temporaries in the library's
per-device scratch array) against the allocating entry point: the same
kernels on the same inputs, so kept dimensions, truncation error and the
packed factors must agree bit for bit.  Two calls in a row, the second on a
smaller wavefunction (the scratch keeps the first call's contents), then the
larger one again; a wavefunction whose temporaries exceed the scratch is
refused with DMRG_ENOMEM; the results are also held to the oracle's
truncation error."""
import numpy as np
import pytest
import torch

from oracle.heff import layout_of
from oracle.svd import svd_truncate as oracle_svd
from tests.conftest import tiny_problem

pytestmark = pytest.mark.gpu


def _l24():
    from synth.problem import WORKLOADS, make_problem
    w = WORKLOADS["l24_d1024"]
    return make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], max_pairs_per_group=1)


def _used(prob, kept):
    """Doubles written to U, S and Vt for the kept dimensions."""
    lay = layout_of(prob)
    u = s = v = 0
    for a in lay.partner:
        k = int(kept[a])
        u += int(lay.Ld[a]) * k
        s += k
        v += k * int(lay.Rd[lay.partner[a]])
    return u, s, v


def _run(ctx, prob, noalloc, keep):
    from paper_2407_07411_amd.heff import svd_truncate
    psi = prob.psi.to("cuda")
    return svd_truncate(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, psi, max_keep=keep, noalloc=noalloc)


def test_noalloc_svd_matches_allocating_entry_point():
    from paper_2407_07411_amd.heff import Context
    ctx = Context(0)
    big = _l24()
    small = tiny_problem(seed=3, D=12, two_sz=2, pairs=2)
    for prob, keep in ((big, 700), (small, 9), (big, 1024)):
        print("case noalloc", layout_of(prob).total, keep, flush=True)
        ref = _run(ctx, prob, False, keep)
        got = _run(ctx, prob, True, keep)
        torch.cuda.synchronize()
        assert np.array_equal(ref[0], got[0])
        # the factors are packed per left sector; only that prefix is written
        used = _used(prob, ref[0])
        for a, b, n in zip(ref[1:4], got[1:4], used):
            assert torch.equal(a[:n], b[:n])
        assert ref[4] == got[4]
        lay = layout_of(prob)
        parts, err_o = oracle_svd(lay, prob.psi.numpy(), keep)
        assert int(np.sum(got[0])) == sum(p[1].size for p in parts.values())
        assert abs(got[4] - err_o) <= 1e-10 * max(1.0, err_o)


def test_noalloc_svd_refuses_oversized_input():
    from paper_2407_07411_amd._lib import DmrgError
    from paper_2407_07411_amd.heff import Context, svd_truncate
    from synth.sectors import bond_sectors
    from synth.problem import WORKLOADS
    w = WORKLOADS["cas63_58_d4096"]
    Lq, Ld, Rq, Rd, Q = bond_sectors(w["L"], w["n_elec"], w["two_sz"], w["D"])
    ctx = Context(0)
    from paper_2407_07411_amd.heff import Basis, wfn_layout
    _, _, total = wfn_layout(Basis(ctx, Lq, Ld), Basis(ctx, Rq, Rd), Q)
    psi = torch.ones(total, dtype=torch.float64, device="cuda")
    with pytest.raises(DmrgError) as ei:
        svd_truncate(ctx, Lq, Ld, Rq, Rd, Q, psi, max_keep=16, noalloc=True)
    assert ei.value.status == -3
    assert "scratch" in str(ei.value)

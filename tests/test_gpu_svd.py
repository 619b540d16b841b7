"""GPU truncating SVD (block one-sided Jacobi) against the oracle
(LAPACK gesdd per block, same global truncation rule).

Compared: kept dimensions per sector (integers, exact), truncation error,
singular values, the reconstruction U S V^T and the orthonormality of the
factors; singular vectors themselves are gauge (signs, degenerate subspaces)
and are not compared entry by entry."""
import numpy as np
import pytest
import torch

from oracle.heff import layout_of
from oracle.svd import reconstruct, svd_truncate as oracle_svd
from tests.conftest import tiny_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def unpack(prob, kept, U, S, Vt):
    lay = layout_of(prob)
    U, S, Vt = U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy()
    parts = {}
    uo = so = vo = 0
    for a in range(len(prob.Ld)):
        k = int(kept[a])
        if a not in lay.partner:
            assert k == 0
            continue
        m, n = int(prob.Ld[a]), int(prob.Rd[lay.partner[a]])
        parts[a] = (U[uo:uo + m * k].reshape(m, k), S[so:so + k], Vt[vo:vo + k * n].reshape(k, n))
        uo += m * k
        so += k
        vo += k * n
    return parts


def _l24_psi():
    from synth.problem import WORKLOADS, make_problem
    w = WORKLOADS["l24_d1024"]
    return make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], max_pairs_per_group=1)


CASES = [("tiny", dict(seed=7, D=12), 10**9), ("tiny", dict(seed=8, D=12), 9),
         ("tiny", dict(seed=9, L=10, n_elec=9, two_sz=1, D=24), 30),
         ("l24", None, 1024), ("l24", None, 256)]


@pytest.mark.parametrize("kind,kw,keep", CASES)
def test_svd_truncate_matches_oracle(ctx, kind, kw, keep):
    from paper_2407_07411_amd.heff import svd_truncate
    print("case", kind, kw, keep, flush=True)
    prob = tiny_problem(**kw) if kind == "tiny" else _l24_psi()
    lay = layout_of(prob)
    psi = prob.psi.numpy()
    ref, ref_err = oracle_svd(lay, psi, keep)
    kept, U, S, Vt, err = svd_truncate(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q,
                                       prob.psi.to("cuda"), keep)
    for a in range(len(prob.Ld)):
        assert int(kept[a]) == (len(ref[a][1]) if a in ref else 0)
    assert abs(err - ref_err) <= 1e-13 + 1e-11 * ref_err
    parts = unpack(prob, kept, U, S, Vt)
    y, yr = reconstruct(lay, parts), reconstruct(lay, ref)
    assert np.linalg.norm(y - yr) <= 1e-12 * np.linalg.norm(yr)
    for a, (u, s, vt) in parts.items():
        assert np.allclose(s, ref[a][1], rtol=0, atol=1e-13)
        if len(s):
            assert np.abs(u.T @ u - np.eye(len(s))).max() < 1e-12
            assert np.abs(vt @ vt.T - np.eye(len(s))).max() < 1e-12

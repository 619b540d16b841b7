"""Pins of the oracle's Davidson, SVD truncation and adjoint.

* Davidson: lowest eigenvalue equals dense `eigh` of the brute-force matrix,
  with and without restarts;
* SVD truncation: exact reconstruction without truncation, Eckart-Young
  (||Psi - Psi_D||_F^2 equals the discarded weight), global ordering;
* adjoint: the Euler identities of a bilinear map, and central finite
  differences along random directions.
"""
import numpy as np
import pytest
import torch

from oracle.davidson import davidson
from oracle.grad import heff_adjoint
from oracle.heff import heff_apply, heff_dense, heff_diag, layout_of
from oracle.svd import reconstruct, svd_truncate
from tests.conftest import tiny_problem, with_one_sided_hc


@pytest.mark.parametrize("max_subspace", [24, 5])
def test_davidson_matches_eigh(max_subspace):
    prob = tiny_problem(seed=6, D=16, pairs=3)
    H = heff_dense(prob)
    e0 = np.linalg.eigvalsh(H)[0]
    res = davidson(lambda v: heff_apply(prob, v), heff_diag(prob),
                   x0=prob.psi.numpy(), tol=1e-9, max_subspace=max_subspace)
    assert res["converged"]
    assert abs(res["energy"] - e0) < 1e-10
    x = res["x"]
    assert np.linalg.norm(H @ x - res["energy"] * x) <= 1e-9 * 1.0001


def test_svd_no_truncation_is_exact():
    prob = tiny_problem(seed=7, D=12, pairs=1)
    lay = layout_of(prob)
    psi = prob.psi.numpy()
    parts, err = svd_truncate(lay, psi, max_keep=10**9)
    assert err < 1e-30
    assert np.abs(reconstruct(lay, parts) - psi).max() < 1e-13


@pytest.mark.parametrize("keep", [1, 5, 17])
def test_svd_eckart_young(keep):
    prob = tiny_problem(seed=8, D=12, pairs=1)
    lay = layout_of(prob)
    psi = prob.psi.numpy()
    parts, err = svd_truncate(lay, psi, max_keep=keep)
    assert sum(len(S) for (_, S, _) in parts.values()) == keep
    diff = reconstruct(lay, parts) - psi
    assert abs(diff @ diff - err) < 1e-13
    # the kept values are the global top-`keep`
    allS = np.sort(np.concatenate([np.linalg.svd(lay.block(psi, a), compute_uv=False) for a in lay.partner]))[::-1]
    kept = np.sort(np.concatenate([S for (_, S, _) in parts.values()]))[::-1]
    assert np.allclose(kept, allS[:keep], rtol=0, atol=1e-14)
    assert abs(err - (allS[keep:] ** 2).sum()) < 1e-13


def _dot(a, b):
    return float(np.dot(np.ravel(a), np.ravel(b)))


@pytest.mark.parametrize("one_sided_hc", [False, True])
def test_adjoint_euler_identities(one_sided_hc):
    prob = tiny_problem(seed=9, D=10, pairs=3)
    if one_sided_hc:
        prob = with_one_sided_hc(prob, seed=9)
    lay = layout_of(prob)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(lay.total)
    ybar = rng.standard_normal(lay.total)
    y = heff_apply(prob, psi)
    pb, gL, gR = heff_adjoint(prob, psi, ybar)
    # f = <ybar, H psi> is linear in psi: <psibar, psi> = f
    assert abs(_dot(pb, psi) - _dot(ybar, y)) < 1e-12 * max(1, abs(_dot(ybar, y)))
    # linear in the left pool for terms with a left op, same for the right
    yl = heff_apply(prob, psi, terms=[t for t in prob.terms if t.one_sided != 2])
    yr = heff_apply(prob, psi, terms=[t for t in prob.terms if t.one_sided != 1])
    lp, rp = prob.left_pool.numpy(), prob.right_pool.numpy()
    assert abs(_dot(gL, lp) - _dot(ybar, yl)) < 1e-12 * max(1, abs(_dot(ybar, yl)))
    assert abs(_dot(gR, rp) - _dot(ybar, yr)) < 1e-12 * max(1, abs(_dot(ybar, yr)))
    # psibar is H^T ybar
    assert np.abs(pb - heff_dense(prob).T @ ybar).max() < 1e-12


@pytest.mark.parametrize("one_sided_hc", [False, True])
def test_adjoint_central_differences(one_sided_hc):
    prob = tiny_problem(seed=10, D=8, pairs=2)
    if one_sided_hc:
        prob = with_one_sided_hc(prob, seed=10)
    lay = layout_of(prob)
    rng = np.random.default_rng(2)
    psi = rng.standard_normal(lay.total)
    ybar = rng.standard_normal(lay.total)
    pb, gL, gR = heff_adjoint(prob, psi, ybar)
    h = 1e-6
    lp, rp = prob.left_pool.numpy(), prob.right_pool.numpy()

    def f(psi_, lp_, rp_):
        return _dot(ybar, heff_apply(prob, psi_, left_pool=torch.from_numpy(lp_), right_pool=torch.from_numpy(rp_)))

    for _ in range(3):
        dpsi = rng.standard_normal(psi.size)
        dl = rng.standard_normal(lp.size)
        dr = rng.standard_normal(rp.size)
        fd = (f(psi + h * dpsi, lp, rp) - f(psi - h * dpsi, lp, rp)) / (2 * h)
        assert abs(fd - _dot(pb, dpsi)) < 1e-7 * max(1, abs(fd))
        fd = (f(psi, lp + h * dl, rp) - f(psi, lp - h * dl, rp)) / (2 * h)
        assert abs(fd - _dot(gL, dl)) < 1e-7 * max(1, abs(fd))
        fd = (f(psi, lp, rp + h * dr) - f(psi, lp, rp - h * dr)) / (2 * h)
        assert abs(fd - _dot(gR, dr)) < 1e-7 * max(1, abs(fd))


def test_rayleigh_gradient_vanishes_at_eigenvector():
    prob = tiny_problem(seed=11, D=8, pairs=2)
    H = heff_dense(prob)
    w, U = np.linalg.eigh(H)
    x = U[:, 0]
    # grad of E = x^T H x / x^T x is 2 (H x - E x) / x^T x, via the adjoint
    pb, _, _ = heff_adjoint(prob, x, x)
    g = 2 * (0.5 * (pb + heff_apply(prob, x)) - w[0] * x)
    assert np.linalg.norm(g) < 1e-10

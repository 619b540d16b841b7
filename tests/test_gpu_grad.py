"""Hand-written adjoint behind torch.autograd.Function on the L=24, D=1024
setup (reduced term list, full shapes): gradients of psi and of both operator
pools against the oracle gradient, central finite differences with step
1e-6 along random directions, and the Rayleigh-quotient gradient."""
import numpy as np
import pytest
import torch

from oracle.grad import heff_adjoint
from tests.test_gpu_heff import _l24, gpu_heff, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


@pytest.fixture(scope="module")
def prob():
    return _l24(1)


def test_autograd_matches_oracle(ctx, prob):
    from paper_2407_07411_amd.heff import HeffApply
    h = gpu_heff(ctx, prob)
    rng = np.random.default_rng(11)
    w = torch.from_numpy(rng.standard_normal(h.size)).cuda()
    psi = prob.psi.to("cuda").clone().requires_grad_(True)
    lp = h.left_pool.requires_grad_(True)
    rp = h.right_pool.requires_grad_(True)
    y = HeffApply.apply(psi, lp, rp, h)
    (w * y).sum().backward()
    pb, gl, gr = heff_adjoint(prob, prob.psi.numpy(), w.cpu().numpy())
    assert rel(psi.grad.cpu().numpy(), pb) <= 1e-12
    assert rel(lp.grad.cpu().numpy(), gl) <= 1e-12
    assert rel(rp.grad.cpu().numpy(), gr) <= 1e-12
    lp.requires_grad_(False)
    rp.requires_grad_(False)


def test_central_differences(ctx, prob):
    h = gpu_heff(ctx, prob)
    rng = np.random.default_rng(12)
    n = h.size
    w = torch.from_numpy(rng.standard_normal(n)).cuda()
    psi = prob.psi.to("cuda").clone()
    gp = torch.zeros_like(psi)
    gl = torch.zeros_like(h.left_pool)
    gr = torch.zeros_like(h.right_pool)
    h.adjoint(psi, w, gp, gl, gr)
    step = 1e-6

    def f():
        return float(torch.dot(w, h.apply(psi)))

    for _ in range(2):
        for grad, target in ((gp, psi), (gl, h.left_pool), (gr, h.right_pool)):
            d = torch.from_numpy(rng.standard_normal(target.numel())).cuda()
            target.add_(step * d)
            fp = f()
            target.sub_(2 * step * d)
            fm = f()
            target.add_(step * d)
            fd = (fp - fm) / (2 * step)
            an = float(torch.dot(grad, d))
            # bilinear loss: no truncation error, rounding ~ eps * |f| / step
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def test_rayleigh_quotient_gradient(ctx, prob):
    from paper_2407_07411_amd.heff import HeffApply
    h = gpu_heff(ctx, prob)
    psi = prob.psi.to("cuda").clone().requires_grad_(True)
    y = HeffApply.apply(psi, h.left_pool, h.right_pool, h)
    E = torch.dot(psi, y) / torch.dot(psi, psi)
    E.backward()
    with torch.no_grad():
        x = psi.detach()
        hx = h.apply(x)
        e = float(torch.dot(x, hx) / torch.dot(x, x))
        ref = 2 * (hx - e * x) / torch.dot(x, x)
    assert rel(psi.grad.cpu().numpy(), ref.cpu().numpy()) <= 1e-10

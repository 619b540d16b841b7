"""The L=24, D=1024 middle bond with its full term list (1226 terms: every
class of the normal/complementary operator split with its hermitian-conjugate
partners; 94 enlarged sectors of 1..209 rows), in the default launch
configuration (tile rule, workspace, K cut):

* forward H_eff psi against the oracle, ||dy|| <= 1e-12 ||y||;
* backward through torch.autograd.Function (psi, left pool, right pool,
  intermediates recomputed) against the oracle gradient at 1e-12, and
  central finite differences with step 1e-6 along random directions of psi
  and of both pools.
"""
import numpy as np
import pytest
import torch

from oracle.grad import heff_adjoint
from oracle.heff import heff_apply
from tests.test_gpu_heff import _l24, gpu_heff, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


@pytest.fixture(scope="module")
def prob():
    p = _l24(None)
    assert len(p.terms) == 626 and sum(1 + t.hc for t in p.terms) == 1226
    return p


def test_forward_all_terms(ctx, prob):
    print("case l24_d1024 all terms forward", flush=True)
    h = gpu_heff(ctx, prob)
    y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    assert rel(y, heff_apply(prob)) <= 1e-12


def test_backward_all_terms(ctx, prob):
    from paper_2407_07411_amd.heff import HeffApply
    print("case l24_d1024 all terms backward", flush=True)
    h = gpu_heff(ctx, prob)
    rng = np.random.default_rng(31)
    w = torch.from_numpy(rng.standard_normal(h.size)).cuda()
    psi = prob.psi.to("cuda").clone().requires_grad_(True)
    lp = h.left_pool.requires_grad_(True)
    rp = h.right_pool.requires_grad_(True)
    y = HeffApply.apply(psi, lp, rp, h)
    (w * y).sum().backward()
    lp.requires_grad_(False)
    rp.requires_grad_(False)
    pb, gl, gr = heff_adjoint(prob, prob.psi.numpy(), w.cpu().numpy())
    assert rel(psi.grad.cpu().numpy(), pb) <= 1e-12
    assert rel(lp.grad.cpu().numpy(), gl) <= 1e-12
    assert rel(rp.grad.cpu().numpy(), gr) <= 1e-12
    # central differences of the bilinear loss <w, H psi> (no truncation
    # error; rounding ~ eps |f| / step)
    step = 1e-6
    x = psi.detach()

    def f():
        return float(torch.dot(w, h.apply(x)))

    for grad, target in ((psi.grad, x), (lp.grad, h.left_pool), (rp.grad, h.right_pool)):
        d = torch.from_numpy(rng.standard_normal(target.numel())).cuda()
        target.add_(step * d)
        fp = f()
        target.sub_(2 * step * d)
        fm = f()
        target.add_(step * d)
        fd = (fp - fm) / (2 * step)
        an = float(torch.dot(grad, d))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)

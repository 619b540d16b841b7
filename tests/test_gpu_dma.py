"""The FP64 kernels that load operand tiles straight into LDS (selected with
DMRG_HEFF_DMA: 1 = two-deep K-tile ring, 2 = three-deep ring for 64x128
tiles, 3 = 128x128 tiles for large problems) against the register-staged
kernels: every output element is summed in the same order, so the matvec
and the adjoint must agree bit for bit; they are also held to the oracle at
1e-12.  Cases: tiny problems (ragged sectors of 1..6 rows, every term class,
one-sided hc terms), the L=24, D=1024 middle bond (reduced term list; odd
and even K lengths, partial K tiles of every length, both operand layouts),
with several workspace waves and cut K sums."""
import numpy as np
import pytest
import torch

from oracle.heff import heff_apply
from tests.conftest import tiny_problem, with_one_sided_hc
from tests.test_gpu_heff import _l24, rel

pytestmark = pytest.mark.gpu

MODES = ["1", "2", "3"]


def _plan(prob, mode, monkeypatch):
    from paper_2407_07411_amd.heff import Context, Heff
    monkeypatch.setenv("DMRG_HEFF_DMA", mode)
    ctx = Context(0)
    h = Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool.to("cuda"),
             prob.right_pool.to("cuda"))
    return ctx, h


def _apply_and_adjoint(prob, mode, monkeypatch):
    ctx, h = _plan(prob, mode, monkeypatch)
    x = prob.psi.to("cuda")
    y = h.apply(x).clone()
    yb = torch.from_numpy(np.random.default_rng(7).standard_normal(h.size)).cuda()
    gp = torch.zeros_like(x)
    gl = torch.zeros_like(h.left_pool)
    gr = torch.zeros_like(h.right_pool)
    h.adjoint(x, yb, gp, gl, gr)
    torch.cuda.synchronize()
    return y, gp, gl, gr


CASES = {
    "tiny": lambda: tiny_problem(seed=2, D=8, pairs=3),
    "tiny_hc": lambda: with_one_sided_hc(tiny_problem(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3), seed=4),
    "l24": lambda: _l24(2),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("mode", MODES)
def test_lds_load_kernels_bit_identical(name, mode, monkeypatch):
    print("case dma", name, mode, flush=True)
    prob = CASES[name]()
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    monkeypatch.setenv("DMRG_HEFF_KCHUNK", "300")
    ref = _apply_and_adjoint(prob, "0", monkeypatch)
    got = _apply_and_adjoint(prob, mode, monkeypatch)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    assert rel(got[0].cpu().numpy(), heff_apply(prob)) <= 1e-12

"""GPU pins of the plan's bookkeeping and of the hermitian-conjugate rule for
one-sided terms, through the C ABI.

* The metric numerator: the library's algorithmic FLOP count (every
  (term, block) pair at its cheaper association, one-sided pairs one GEMM)
  and byte count (every used stored block once, psi read, y written) equal
  the oracle's counts exactly, on tiny problems, the full L=24, D=1024 term
  list and the physical L=8 centre bond.
* One-sided terms flagged hc = 1 also apply their transposed block (the
  effective Hamiltonian of Eq. 2 is hermitian): matvec, diagonal and adjoint
  agree with the oracle at 1e-12 on problems whose one-sided blocks are
  non-symmetric.
* Graph capture needs a caller stream: use_graph on the null stream is
  refused with DMRG_EINVAL.
"""
import numpy as np
import pytest
import torch

from oracle.grad import heff_adjoint
from oracle.heff import count_bytes, count_flops, heff_apply, heff_diag, layout_of
from tests.conftest import tiny_problem, with_one_sided_hc
from tests.test_gpu_heff import _l24, gpu_heff, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def _physical():
    from oracle.physical import physical_problem
    from synth.integrals import integrals
    h_, V = integrals(8, 1001)
    return physical_problem(h_, V, 4, 4, 4)


COUNT_CASES = {
    "tiny": lambda: tiny_problem(seed=2, D=8, pairs=3),
    "tiny_one_sided_hc": lambda: with_one_sided_hc(tiny_problem(seed=3, D=12, two_sz=2, pairs=2), seed=3),
    "l24_d1024_all_terms": lambda: _l24(None),
    "physical_l8_centre": _physical,
}


@pytest.mark.parametrize("name", sorted(COUNT_CASES))
def test_flop_and_byte_counts_equal_oracle(ctx, name):
    print("case counts", name, flush=True)
    prob = COUNT_CASES[name]()
    h = gpu_heff(ctx, prob)
    flops, nbytes = h.flops()
    assert flops == float(count_flops(prob))
    assert nbytes == float(count_bytes(prob))


HC_CASES = [
    dict(seed=1, D=4, pairs=2),
    dict(seed=3, D=12, two_sz=2, pairs=2),
    dict(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3),
]


@pytest.mark.parametrize("kw", HC_CASES)
def test_one_sided_hc_matvec_diag_adjoint(ctx, kw):
    print("case one-sided hc", kw, flush=True)
    prob = with_one_sided_hc(tiny_problem(**kw), seed=kw["seed"])
    assert any(t.one_sided and t.hc for t in prob.terms)
    h = gpu_heff(ctx, prob)
    x = prob.psi.to("cuda")
    y = h.apply(x).cpu().numpy()
    assert rel(y, heff_apply(prob)) <= 1e-12
    d = h.diag().cpu().numpy()
    ref = heff_diag(prob)
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()
    rng = np.random.default_rng(kw["seed"])
    yb = rng.standard_normal(h.size)
    gp = torch.zeros_like(x)
    gl = torch.zeros_like(h.left_pool)
    gr = torch.zeros_like(h.right_pool)
    h.adjoint(x, torch.from_numpy(yb).cuda(), gp, gl, gr)
    pb, rl, rr = heff_adjoint(prob, prob.psi.numpy(), yb)
    assert rel(gp.cpu().numpy(), pb) <= 1e-12
    assert rel(gl.cpu().numpy(), rl) <= 1e-12
    assert rel(gr.cpu().numpy(), rr) <= 1e-12


def test_one_sided_hc_l24(ctx):
    """The same rule at L=24, D=1024 (reduced term list, full shapes)."""
    prob = with_one_sided_hc(_l24(1), seed=24, scale=0.05)
    h = gpu_heff(ctx, prob)
    y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    assert rel(y, heff_apply(prob)) <= 1e-12


def test_graph_on_null_stream_is_refused():
    from paper_2407_07411_amd._lib import DmrgError
    from paper_2407_07411_amd.heff import Context, Heff
    prob = tiny_problem(seed=1, D=4, pairs=2)
    with torch.cuda.stream(torch.cuda.default_stream()):
        c = Context(0)
        assert torch.cuda.current_stream().cuda_stream == 0
        h = Heff(c, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool.to("cuda"),
                 prob.right_pool.to("cuda"))
        h.use_graph(True)
        with pytest.raises(DmrgError) as ei:
            h.apply(prob.psi.to("cuda"))
        assert ei.value.status == -1
        h.use_graph(False)
        y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    assert rel(y, heff_apply(prob)) <= 1e-12

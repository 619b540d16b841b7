"""GPU parity of the SU(2) spin-adapted form (dmrg_heff_create_su2) against
the SU(2) oracle, through the C ABI.

The oracle is pinned on the CPU against the U(1) oracle on the expanded
problem (tests/test_oracle_su2.py).  Here: the reduced matvec at
||Δy||/||y|| <= 1e-12 on tiny problems (every term class, half-integer
spins, several total S) and on a larger one whose reduced blocks span
several 64/128 tiles with ragged tails; the diagonal; the FLOP count; the
layout; Davidson against dense eigh; split precision within its bound; the
adjoint (H^T ybar and a central finite difference of the pool gradients);
the persistent launch bit-identical to the per-phase launches; and the
host-side refusals."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.su2 import count_flops_su2, heff_apply_su2, heff_dense_su2, heff_diag_su2, layout_su2
from synth.su2 import tiny_su2

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def plan(ctx, prob, prec=0):
    from paper_2407_07411_amd.heff import HeffSU2
    return HeffSU2(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool.to("cuda"),
                   prob.right_pool.to("cuda"), prec=prec)


CASES = {
    "s0": dict(seed=1, N=6, two_s=0),
    "s_half": dict(seed=2, N=5, two_s=1),
    "s1": dict(seed=3, N=6, two_s=2),
    "s3_half": dict(seed=4, N=5, two_s=3),
    "s2": dict(seed=5, N=4, two_s=4, n_hi=3, tj_max=2),
    "medium": dict(seed=11, n_lo=2, n_hi=7, tj_max=5, dmax=150, N=9, two_s=1, pairs=3),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = tiny_su2(**CASES[name])
    return _cache[name]


@pytest.mark.parametrize("name", sorted(CASES))
def test_matvec_diag_flops(ctx, name):
    print("case su2", name, flush=True)
    prob = case(name)
    h = plan(ctx, prob)
    x = prob.psi.to("cuda")
    y = h.apply(x).cpu().numpy()
    d = h.diag().cpu().numpy()
    torch.cuda.synchronize()
    assert h.size == layout_su2(prob).total
    assert rel(y, heff_apply_su2(prob)) <= 1e-12
    dref = heff_diag_su2(prob)
    assert np.abs(d - dref).max() <= 1e-13 * max(1.0, np.abs(dref).max())
    assert h.flops()[0] == count_flops_su2(prob)


def test_layout(ctx):
    from paper_2407_07411_amd.heff import wfn_layout_su2
    prob = case("s3_half")
    h = plan(ctx, prob)
    bl, br, bo, total = wfn_layout_su2(h.L, h.R, prob.Q)
    lay = layout_su2(prob)
    assert total == lay.total
    assert [(int(a), int(c)) for a, c in zip(bl, br)] == lay.blocks
    assert [int(o) for o in bo] == [lay.offset[b] for b in lay.blocks]


def test_davidson_lowest_eigenvalue(ctx):
    from paper_2407_07411_amd.heff import davidson
    prob = case("s1")
    w = np.linalg.eigvalsh(heff_dense_su2(prob))
    h = plan(ctx, prob)
    psi = prob.psi.to("cuda").clone()
    r = davidson(h, psi, tol=1e-10, max_iter=200)
    print(r, w[0], flush=True)
    assert r["converged"] and abs(r["energy"] - w[0]) < 1e-9


@pytest.mark.parametrize("prec", [1, 3])
def test_reduced_precision_bound(ctx, prec):
    prob = case("medium")
    h = plan(ctx, prob, prec=prec)
    y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    err = rel(y, heff_apply_su2(prob))
    print("su2 reduced precision", prec, err, flush=True)
    assert 0.0 < err <= 1e-5


def test_adjoint(ctx):
    prob = case("s3_half")
    h = plan(ctx, prob)
    n = h.size
    g = torch.Generator().manual_seed(5)
    x = prob.psi.to("cuda")
    yb = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    pb = torch.zeros_like(x)
    gl = torch.zeros_like(h.left_pool)
    gr = torch.zeros_like(h.right_pool)
    h.adjoint(x, yb, pb, gl, gr)
    torch.cuda.synchronize()
    H = heff_dense_su2(prob)
    assert rel(pb.cpu().numpy(), H.T @ yb.cpu().numpy()) <= 1e-12
    # pool gradients: central difference of <ybar, H(pools) psi> along a random direction
    vl = torch.randn(h.left_pool.numel(), generator=g, dtype=torch.float64)
    vr = torch.randn(h.right_pool.numel(), generator=g, dtype=torch.float64)
    import dataclasses
    eps = 1e-6

    def f(s):
        p = dataclasses.replace(prob, left_pool=prob.left_pool + s * vl, right_pool=prob.right_pool + s * vr)
        return float(np.dot(yb.cpu().numpy(), heff_apply_su2(p)))
    fd = (f(eps) - f(-eps)) / (2 * eps)
    an = float(torch.dot(gl.cpu(), vl) + torch.dot(gr.cpu(), vr))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_persistent_bit_identical(ctx, monkeypatch):
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    monkeypatch.setenv("DMRG_HEFF_KCHUNK", "300")
    prob = case("medium")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    from paper_2407_07411_amd.heff import Context
    with torch.cuda.stream(stream):
        c2 = Context(0)
        h = plan(c2, prob)
        x = prob.psi.to("cuda")
        ref = h.apply(x).clone()
        h.set_persistent(True)
        ys = [h.apply(x).clone() for _ in range(2)]
        h.check()
    torch.cuda.synchronize()
    for y in ys:
        assert torch.equal(y, ref)
    assert rel(ref.cpu().numpy(), heff_apply_su2(prob)) <= 1e-12


def test_refusals(ctx):
    import dataclasses

    from paper_2407_07411_amd._lib import DmrgError
    prob = case("s_half")
    # a block whose output sector breaks N' - N = dn
    t = next(t for t in prob.terms if t.two_k == 2 and not t.one_sided)
    tab = np.asarray(t.left_blocks).copy()
    Lq = np.asarray(prob.Lq)
    o, a, _ = tab[0].tolist()
    o2 = next(i for i in range(len(Lq)) if Lq[i][0] != Lq[o][0])
    tab[0, 0] = o2
    terms = [dataclasses.replace(x, left_blocks=tab) if x is t else x for x in prob.terms]
    with pytest.raises(DmrgError) as e:
        plan(ctx, dataclasses.replace(prob, terms=terms))
    assert e.value.status == -2
    # a one-sided term that is not a scalar
    t1 = next(t for t in prob.terms if t.one_sided == 1)
    terms = [dataclasses.replace(x, two_k=2) if x is t1 else x for x in prob.terms]
    with pytest.raises(DmrgError) as e:
        plan(ctx, dataclasses.replace(prob, terms=terms))
    assert e.value.status == -2
    # 2j < 0 in a basis
    Lq2 = np.asarray(prob.Lq).copy()
    Lq2[0, 1] = -1
    with pytest.raises(DmrgError) as e:
        plan(ctx, dataclasses.replace(prob, Lq=Lq2))
    assert e.value.status == -1


def test_l24_d512_every_term(ctx):
    """The L=24, 24-electron singlet bond at D=512 multiplets with every
    operator pair of every class (572 terms, reduced blocks up to 151
    multiplets, 1.3 GB of pools): the shape class of the U(1) L=24 case."""
    from synth.su2 import make_workload_su2
    print("case su2_l24_d512", flush=True)
    prob = make_workload_su2("su2_l24_d512")
    h = plan(ctx, prob)
    y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    torch.cuda.synchronize()
    assert rel(y, heff_apply_su2(prob)) <= 1e-12
    assert h.flops()[0] == count_flops_su2(prob)

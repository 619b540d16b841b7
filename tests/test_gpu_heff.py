"""GPU parity of the H_eff matvec, its diagonal and its adjoint against the
CPU FP64 oracle, through the C ABI.

Tolerance: ||y_gpu - y_oracle||_2 <= 1e-12 ||y_oracle||_2 (norm-wise: the
two sides sum the same products in different orders, so single entries may
cancel).  Sizes: tiny problems (ragged sectors of 1..6 rows) with every term
class, the L=24, D=1024 middle bond with a reduced term list (full shapes,
sectors of 1..209 rows spanning several tiles and ragged tails), and the
physical L=8 centre bond whose pairs come from the real Hamiltonian.
"""
import numpy as np
import pytest
import torch

from oracle.grad import heff_adjoint
from oracle.heff import heff_apply, heff_diag, layout_of
from tests.conftest import tiny_problem

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def gpu_heff(ctx, prob, prec=0):
    from paper_2407_07411_amd.heff import Heff
    lp = prob.left_pool.to("cuda")
    rp = prob.right_pool.to("cuda")
    return Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, lp, rp, prec=prec)


PROBLEMS = [
    dict(seed=1, D=4, pairs=2),
    dict(seed=2, D=8, pairs=3),
    dict(seed=3, D=12, two_sz=2, pairs=2),
    dict(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3),
]


@pytest.mark.parametrize("kw", PROBLEMS)
def test_matvec_tiny(ctx, kw):
    print("case", kw, flush=True)
    prob = tiny_problem(**kw)
    h = gpu_heff(ctx, prob)
    y = h.apply(prob.psi.to("cuda"))
    torch.cuda.synchronize()
    ref = heff_apply(prob)
    assert rel(y.cpu().numpy(), ref) <= TOL


def _l24(pairs):
    from synth.problem import WORKLOADS, make_problem
    w = dict(WORKLOADS["l24_d1024"])
    return make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], max_pairs_per_group=pairs)


@pytest.fixture(scope="module")
def l24():
    return _l24(2)


def test_matvec_l24_reduced_terms(ctx, l24):
    print("case l24_d1024 pairs<=2", flush=True)
    h = gpu_heff(ctx, l24)
    y = h.apply(l24.psi.to("cuda")).cpu().numpy()
    ref = heff_apply(l24)
    assert rel(y, ref) <= TOL


@pytest.mark.parametrize("tile", ["32", "64", "128", "1288", "256", "64128"])
def test_matvec_tile_shapes(ctx, l24, tile, monkeypatch):
    print("case tile", tile, flush=True)
    monkeypatch.setenv("DMRG_HEFF_TILE", tile)
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")  # force several waves
    h = gpu_heff(ctx, l24)
    y = h.apply(l24.psi.to("cuda")).cpu().numpy()
    assert rel(y, heff_apply(l24)) <= TOL


def test_diag(ctx, l24):
    h = gpu_heff(ctx, l24)
    d = h.diag().cpu().numpy()
    ref = heff_diag(l24)
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()


def test_deterministic_and_graph_replay(ctx, l24):
    h = gpu_heff(ctx, l24)
    x = l24.psi.to("cuda")
    y0 = h.apply(x).clone()
    y1 = h.apply(x).clone()
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    side.wait_stream(torch.cuda.current_stream())
    ys = []
    with torch.cuda.stream(side):
        h.use_graph(True)
        out = torch.empty_like(x)
        for _ in range(3):
            h.apply(x, out)
            torch.cuda.synchronize()
            ys.append(out.clone())
            out.fill_(1.0)  # eager work between replays
        h.use_graph(False)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    for y in ys:
        assert torch.equal(y, y0)


def test_adjoint(ctx):
    prob = tiny_problem(seed=9, L=10, n_elec=10, D=20, pairs=3)
    h = gpu_heff(ctx, prob)
    rng = np.random.default_rng(5)
    lay = layout_of(prob)
    psi = rng.standard_normal(lay.total)
    ybar = rng.standard_normal(lay.total)
    pb, gl, gr = heff_adjoint(prob, psi, ybar)
    dpsi = torch.from_numpy(psi).cuda()
    dyb = torch.from_numpy(ybar).cuda()
    gp = torch.zeros_like(dpsi)
    gL = torch.zeros_like(h.left_pool)
    gR = torch.zeros_like(h.right_pool)
    h.adjoint(dpsi, dyb, gp, gL, gR)
    torch.cuda.synchronize()
    assert rel(gp.cpu().numpy(), pb) <= TOL
    assert rel(gL.cpu().numpy(), gl) <= TOL
    assert rel(gR.cpu().numpy(), gr) <= TOL
    # accumulation semantics: a second call doubles the result
    h.adjoint(dpsi, dyb, gp, None, None)
    assert rel(gp.cpu().numpy(), 2 * pb) <= TOL


def test_physical_centre_matvec(ctx):
    from oracle.physical import physical_problem
    from synth.integrals import integrals
    h_, V = integrals(8, 1001)
    prob = physical_problem(h_, V, 4, 4, 4)
    lay = layout_of(prob)
    x = np.random.default_rng(3).standard_normal(lay.total)
    g = gpu_heff(ctx, prob)
    y = g.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, heff_apply(prob, x)) <= TOL


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_autotune_keeps_results(ctx, l24, prec):
    """FP64 and FP32 operands: tile shapes change only the tiling, not any
    element's summation order (same K sequence, same 4-deep MFMA steps, FP32
    partials flushed every 128 K values), so the autotuned plan reproduces the
    default plan bit for bit.  Split precision: the BF16 MFMAs sum 16 K values
    in an order set by the K tile depth, which differs between shapes, so the
    tuned plan is held to the split bound instead."""
    print("case autotune prec", prec, flush=True)
    h = gpu_heff(ctx, l24, prec=prec)
    x = l24.psi.to("cuda")
    y0 = h.apply(x).clone()
    h.autotune(x, reps=2)
    y1 = h.apply(x)
    torch.cuda.synchronize()
    ref = heff_apply(l24)
    if prec == 1:
        assert rel(y1.cpu().numpy(), ref) <= 1e-5
    else:
        assert torch.equal(y0, y1)
        assert rel(y1.cpu().numpy(), ref) <= (TOL if prec == 0 else 1e-5)


@pytest.mark.parametrize("kchunk", ["64", "700"])
def test_split_k_sums(ctx, l24, kchunk, monkeypatch):
    """Output sums cut into K parts (partials reduced in part order) agree
    with the oracle, and repeat bit for bit."""
    print("case kchunk", kchunk, flush=True)
    monkeypatch.setenv("DMRG_HEFF_KCHUNK", kchunk)
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "8")
    h = gpu_heff(ctx, l24)
    x = l24.psi.to("cuda")
    y0 = h.apply(x).clone()
    y1 = h.apply(x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    assert rel(y0.cpu().numpy(), heff_apply(l24)) <= TOL
    # adjoint programs cut their long sums the same way
    rng = np.random.default_rng(4)
    yb = rng.standard_normal(h.size)
    gp = torch.zeros_like(x)
    h.adjoint(x, torch.from_numpy(yb).cuda(), gp, None, None)
    pb, _, _ = heff_adjoint(l24, l24.psi.numpy(), yb)
    assert rel(gp.cpu().numpy(), pb) <= TOL


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_two_stream_phases_match_serial(l24, prec, monkeypatch):
    """On a caller stream, each phase runs its smaller tile shapes on a side
    stream next to the largest one, and K-split reductions run next to the
    following intermediate phase: with many waves, long sums cut in parts and
    every tile shape in use, the result equals the one-stream order bit for
    bit (and the oracle), eagerly and from a replayed graph."""
    from paper_2407_07411_amd.heff import Context, Heff
    print("case two-stream prec", prec, flush=True)
    monkeypatch.setenv("DMRG_HEFF_KCHUNK", "300")
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    ys = []
    with torch.cuda.stream(stream):
        c = Context(0)
        x = l24.psi.to("cuda")
        for serial in ("1", "0"):
            monkeypatch.setenv("DMRG_HEFF_SERIAL", serial)
            h = Heff(c, l24.Lq, l24.Ld, l24.Rq, l24.Rd, l24.Q, l24.terms, l24.left_pool.to("cuda"),
                     l24.right_pool.to("cuda"), prec=prec)
            ys.append(h.apply(x).clone())
            if serial == "0":
                ys.append(h.apply(x).clone())
                h.use_graph(True)
                for _ in range(3):
                    ys.append(h.apply(x).clone())
                h.use_graph(False)
    torch.cuda.synchronize()
    for y in ys[1:]:
        assert torch.equal(ys[0], y)
    if prec == 0:
        assert rel(ys[0].cpu().numpy(), heff_apply(l24)) <= TOL

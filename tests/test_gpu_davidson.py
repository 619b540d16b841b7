"""GPU Davidson against the oracle: lowest eigenvalue of H_eff to <= 1e-8
(FP64 path), with and without restarts, eager and hipGraph-replayed, and the
FCI energy at the L=8 centre bond."""
import numpy as np
import pytest
import torch

from oracle.davidson import davidson as oracle_davidson
from oracle.heff import heff_apply, heff_dense, heff_diag, layout_of
from tests.conftest import tiny_problem
from tests.test_gpu_heff import gpu_heff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


@pytest.mark.parametrize("max_subspace,keep", [(24, 2), (5, 1), (6, 3)])
def test_davidson_tiny_matches_eigh(ctx, max_subspace, keep):
    from paper_2407_07411_amd.heff import davidson
    prob = tiny_problem(seed=6, D=16, pairs=3)
    e0 = np.linalg.eigvalsh(heff_dense(prob))[0]
    h = gpu_heff(ctx, prob)
    psi = prob.psi.to("cuda").clone()
    res = davidson(h, psi, tol=1e-9, max_subspace=max_subspace, restart_keep=keep)
    print(res, flush=True)
    assert res["converged"]
    assert abs(res["energy"] - e0) < 1e-8
    x = psi.cpu().numpy()
    assert abs(np.linalg.norm(x) - 1) < 1e-12
    r = heff_apply(prob, x) - res["energy"] * x
    assert np.linalg.norm(r) < 1e-8


def test_davidson_graph_matches_eager(ctx):
    from paper_2407_07411_amd.heff import davidson
    prob = tiny_problem(seed=7, L=10, n_elec=10, D=24, pairs=3)
    h = gpu_heff(ctx, prob)
    p1 = prob.psi.to("cuda").clone()
    r1 = davidson(h, p1, tol=1e-9, max_subspace=8, restart_keep=2)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        p2 = prob.psi.to("cuda").clone()
        r2 = davidson(h, p2, tol=1e-9, max_subspace=8, restart_keep=2, use_graph=True)
    torch.cuda.synchronize()
    assert r1["converged"] and r2["converged"]
    assert r1["energy"] == r2["energy"] and r1["iters"] == r2["iters"]
    assert torch.equal(p1, p2)


def test_davidson_l24_reduced_vs_oracle(ctx):
    from paper_2407_07411_amd.heff import davidson
    from tests.test_gpu_heff import _l24
    prob = _l24(1)
    # start from the unit vector at the lowest diagonal element (a random
    # start converges far more slowly on these synthetic spectra)
    ref = oracle_davidson(lambda v: heff_apply(prob, v), heff_diag(prob), x0=None, tol=1e-8)
    h = gpu_heff(ctx, prob)
    psi = prob.psi.to("cuda").clone()
    res = davidson(h, psi, tol=1e-8, start_from_diag=True)
    print(res, ref["energy"], ref["iters"], flush=True)
    assert res["converged"] and ref["converged"]
    assert abs(res["energy"] - ref["energy"]) < 1e-8


def test_davidson_l8_centre_is_fci(ctx):
    from oracle.fci import fci_energy
    from oracle.physical import physical_problem
    from paper_2407_07411_amd.heff import davidson
    from synth.integrals import integrals
    h_, V = integrals(8, 1001)
    prob = physical_problem(h_, V, 4, 4, 4)
    e_fci = fci_energy(h_, V, 4, 4)
    g = gpu_heff(ctx, prob)
    x0 = np.random.default_rng(8).standard_normal(layout_of(prob).total)
    psi = torch.from_numpy(x0).cuda()
    res = davidson(g, psi, tol=1e-8)
    print(res, e_fci, flush=True)
    assert res["converged"]
    assert abs(res["energy"] - e_fci) < 1e-8


def test_davidson_step_api(ctx):
    import ctypes
    from paper_2407_07411_amd import _lib
    prob = tiny_problem(seed=6, D=16, pairs=3)
    e0 = np.linalg.eigvalsh(heff_dense(prob))[0]
    h = gpu_heff(ctx, prob)
    psi = prob.psi.to("cuda").clone()
    L = _lib.lib()
    opts = _lib.DavOpts(100, 10, 2, 0, 1e-9, 0, 0)
    d = ctypes.c_void_p()
    _lib.check(L.dmrg_davidson_create(h.h, ctypes.byref(opts), ctypes.c_void_p(psi.data_ptr()), ctypes.byref(d)))
    res = _lib.DavResult()
    last = None
    for _ in range(100):
        _lib.check(L.dmrg_davidson_step(d, ctypes.byref(res)))
        last = res.residual
        if res.converged:
            break
    out = torch.empty_like(psi)
    _lib.check(L.dmrg_davidson_vector(d, ctypes.c_void_p(out.data_ptr())))
    torch.cuda.synchronize()
    L.dmrg_davidson_destroy(d)
    assert res.converged and last <= 1e-9
    assert abs(res.energy - e0) < 1e-8


@pytest.mark.parametrize("use_graph", [0, 1])
def test_step_stall_keeps_last_iteration(use_graph):
    """A 21-dimensional problem with tolerance 0: once the subspace spans the
    whole space the next correction vanishes.  The step that finds it (one
    launch sequence: correction, matvec, Rayleigh-Ritz) reports
    DMRG_ENOCONV and leaves the energy, the residual and the Ritz vector of
    the last complete iteration, which by then is the exact ground state."""
    import ctypes

    from paper_2407_07411_amd import _lib
    from paper_2407_07411_amd.heff import Context
    print("case stall", use_graph, flush=True)
    prob = tiny_problem(seed=1, D=4, pairs=2)
    Hd = heff_dense(prob)
    w, _ = np.linalg.eigh(Hd)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        ctx = Context(0)
        h = gpu_heff(ctx, prob)
        psi = prob.psi.to("cuda").clone()
        L = _lib.lib()
        opts = _lib.DavOpts(200, 24, 2, use_graph, 0.0, 0, 0)
        d = ctypes.c_void_p()
        _lib.check(L.dmrg_davidson_create(h.h, ctypes.byref(opts), ctypes.c_void_p(psi.data_ptr()),
                                          ctypes.byref(d)))
        res = _lib.DavResult()
        history = []
        st = 0
        for _ in range(60):
            st = L.dmrg_davidson_step(d, ctypes.byref(res))
            if st != 0:
                break
            history.append((res.energy, res.residual, res.iters))
        msg = L.dmrg_last_error().decode()
        out = torch.empty_like(psi)
        _lib.check(L.dmrg_davidson_vector(d, ctypes.c_void_p(out.data_ptr())))
        torch.cuda.synchronize()
        L.dmrg_davidson_destroy(d)
    assert st == -5 and "vanished" in msg, (st, msg)
    assert len(history) <= 23
    assert (res.energy, res.residual, res.iters) == history[-1]
    assert abs(res.energy - w[0]) < 1e-10
    x = out.cpu().numpy()
    assert np.linalg.norm(Hd @ x - w[0] * x) < 1e-8

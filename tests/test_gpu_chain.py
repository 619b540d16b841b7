"""Two-site DMRG sweeps through the library (operator blocks grown by the
library, renormalised O <- U^T O U as grouped GEMMs on the GPU, H_eff,
Davidson and SVD truncation on the GPU) against the FCI oracle; the device
renormalisation against the host one; the energy gradient with respect to
h through the library's build against the FCI one-particle density matrix.

L=6 with D=64: every cut of the chain has Schmidt rank <= 4^3 = 64, so after
two sweeps every two-site step reproduces E_FCI.  L=8 with D=64 (8 electrons,
Sz=0): the centre step (orbitals 3, 4) holds the whole FCI space once the
blocks [0,3) and [5,8) keep their 64 states, so its energy is E_FCI; every
other step is variational."""
import numpy as np
import pytest

from oracle.fci import fci_energy
from synth.integrals import integrals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def run_sweeps(ch, n):
    out = []
    for _ in range(n):
        out += ch.sweep(+1, tol=1e-9)
        out += ch.sweep(-1, tol=1e-9)
    return out


def test_l6_sweeps_reach_fci(ctx):
    from paper_2407_07411_amd.chain import Chain
    h, V = integrals(6, 21)
    e_fci = fci_energy(h, V, 3, 3, dense=True)
    ch = Chain(ctx, h, V, 6, 0, D=64, seed=5)
    steps = run_sweeps(ch, 2)
    print([round(s["energy"] - e_fci, 12) for s in steps], flush=True)
    for s in steps:
        assert s["energy"] >= e_fci - 1e-9
    last = steps[-(2 * 5):]
    assert max(abs(s["energy"] - e_fci) for s in last) < 1e-7


def test_l8_centre_step_is_fci(ctx):
    from paper_2407_07411_amd.chain import Chain
    h, V = integrals(8, 1001)
    e_fci = fci_energy(h, V, 4, 4)
    ch = Chain(ctx, h, V, 8, 0, D=64, seed=7)
    steps = run_sweeps(ch, 2)
    for s in steps:
        print(s["site"], round(s["energy"] - e_fci, 10), s["trunc_err"], s["converged"], s["iters"],
              s["residual"], flush=True)
    for s in steps:
        assert s["converged"]
        assert s["energy"] >= e_fci - 1e-9
    centre = [s for s in steps if s["site"] == 3]
    assert abs(centre[-1]["energy"] - e_fci) < 1e-8


def _pools_close(a, b, tol=1e-12):
    assert np.array_equal(a.Lq, b.Lq) and np.array_equal(a.Ld, b.Ld)
    assert np.array_equal(a.Rq, b.Rq) and np.array_equal(a.Rd, b.Rd)
    assert len(a.terms) == len(b.terms)
    for ta, tb in zip(a.terms, b.terms):
        for x, y in ((ta.left_off, tb.left_off), (ta.right_off, tb.right_off)):
            assert (x is None) == (y is None) and (x is None or np.array_equal(x, y))
    for pa, pb in ((a.left_pool, b.left_pool), (a.right_pool, b.right_pool)):
        assert pa.shape == pb.shape
        assert np.abs(pa - pb).max() <= tol * max(1.0, np.abs(pb).max())


def test_device_renormalisation_matches_host(ctx, monkeypatch):
    """Right blocks built at creation (random isometries onto D states, every
    operator renormalised) and the left block renormalised after one sweep
    step: device and host renormalisation give the same operators to
    rounding (creation: pools compared entry by entry; after the step, whose
    SVD factors are gauge-dependent: the spectrum of the next H_eff)."""
    from oracle.heff import heff_dense
    from paper_2407_07411_amd.chain import Chain
    h, V = integrals(8, 1001)
    chains = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("DMRG_CHAIN_HOST_RENORM", mode)
        chains[mode] = Chain(ctx, h, V, 8, 0, D=64, seed=7)
    _pools_close(chains["0"].export(0), chains["1"].export(0))
    spectra = {}
    for mode, ch in chains.items():
        monkeypatch.setenv("DMRG_CHAIN_HOST_RENORM", mode)
        ch.step(0, +1, tol=1e-11)
        spectra[mode] = np.linalg.eigvalsh(heff_dense(ch.export(1)))[:8]
    assert np.abs(spectra["0"] - spectra["1"]).max() < 1e-9


@pytest.mark.parametrize("L,na,nb,seed", [(4, 2, 2, 31), (6, 3, 3, 33)])
def test_energy_gradient_through_build_is_rdm1_gpu(ctx, L, na, nb, seed):
    """dE/dh_pq = psi^T H_eff(E_pq, V = 0) psi with every H_eff built by the
    library (full bond dimension: the two-site space is the FCI sector), psi
    from the library's Davidson and every product from its GPU matvec."""
    import torch

    from oracle.fci import fci_rdm1
    from paper_2407_07411_amd.chain import Chain
    from paper_2407_07411_amd.heff import Heff, davidson
    h, V = integrals(L, seed)
    E0, g, gap = fci_rdm1(h, V, na, nb)
    assert gap > 1e-4

    def plan(hh, VV):
        p = Chain(ctx, hh, VV, na + nb, na - nb, D=4 ** L, seed=3).export(0)
        lp = torch.from_numpy(p.left_pool).cuda()
        rp = torch.from_numpy(p.right_pool).cuda()
        return Heff(ctx, p.Lq, p.Ld, p.Rq, p.Rd, p.Q, p.terms, lp, rp), (lp, rp)

    H, keep = plan(h, V)
    psi = torch.from_numpy(np.random.default_rng(1).standard_normal(H.size)).cuda()
    r = davidson(H, psi, tol=1e-11, max_iter=300)
    assert r["converged"] and abs(r["energy"] - E0) < 1e-9
    zero = np.zeros_like(V)
    got = np.zeros((L, L))
    for p in range(L):
        for q in range(L):
            e = np.zeros((L, L))
            e[p, q] = 1.0
            Hpq, k2 = plan(e, zero)
            got[p, q] = float(torch.dot(psi, Hpq.apply(psi)))
    assert np.abs(got - g).max() < 1e-8, np.abs(got - g).max()

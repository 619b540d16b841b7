import os
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def tiny_problem(seed=1, L=8, n_elec=8, two_sz=0, D=8, pairs=2, budget=None, device="cpu"):
    from synth.problem import make_problem
    return make_problem(L, n_elec, two_sz, D, seed, device=device,
                        max_pairs_per_group=pairs, pool_budget_bytes=budget)


@pytest.fixture
def tiny():
    return tiny_problem()


def with_one_sided_hc(prob, seed=0, scale=0.5):
    """The same problem with hc = 1 on its one-sided (H_L (x) 1, 1 (x) H_R)
    terms and their stored blocks made non-symmetric by a seeded random
    perturbation: a dropped hermitian-conjugate partner, or one applied
    without the transpose, changes the operator."""
    import dataclasses

    import numpy as np

    rng = np.random.default_rng(seed)
    lp = prob.left_pool.detach().cpu().clone()
    rp = prob.right_pool.detach().cpu().clone()
    terms = []
    for t in prob.terms:
        if t.one_sided:
            offs, dims, pool = ((t.left_off, prob.Ld, lp) if t.one_sided == 1 else (t.right_off, prob.Rd, rp))
            for s, off in enumerate(np.asarray(offs).tolist()):
                if off < 0:
                    continue
                d = int(dims[s])
                pool[off:off + d * d] += torch.from_numpy(scale * rng.standard_normal(d * d))
            t = dataclasses.replace(t, hc=1)
        terms.append(t)
    dev = prob.left_pool.device
    return dataclasses.replace(prob, terms=terms, left_pool=lp.to(dev), right_pool=rp.to(dev))

import os
import sys

import pytest

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

"""Reduced-precision matvecs and Davidson against the FP64 oracle: split
precision (BF16x3 slices, FP32 accumulation per K chunk, FP64 combine) and
FP32 operands on the FP32 matrix cores (same accumulation; operands rounded
to FP32, 2^-24 relative, like the slices), under the same bound.

Stated bound for the matvec: ||y_split - y||_2 <= 1e-5 ||y||_2.  Derivation:
the slices represent each operand to ~2^-24 relative (FP32 rounding of the
FP64 value plus the slicing), the six kept slice products drop terms of
~2^-24 relative, and an FP32 partial sums at most 2048 K values x 6 products
(the plan cuts split-precision sums every 2048 K values; the
FP64-accumulating kernels flush every 128) before it is added into FP64:
with independent rounding errors the relative error of an output is
~sqrt(12288) x 2^-24 ~ 7e-6, and below 1e-6 where, as here, the terms of a
sum vary in sign and size (aligned worst case: 12288 x 2^-24 ~ 7e-4); the
parity runs see 2e-7 to 9e-7.  Energies: the split phase stalls near the
matvec error and an FP64 tail restarted from its Ritz vector converges to
the FP64 tolerance, so the energy must match the FP64 solve to 1e-8."""
import numpy as np
import pytest
import torch

from oracle.heff import heff_apply, heff_dense
from tests.conftest import tiny_problem
from tests.test_gpu_heff import _l24, gpu_heff, rel

pytestmark = pytest.mark.gpu

SPLIT_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


@pytest.mark.parametrize("prec", ["split", "fp32"])
@pytest.mark.parametrize("kind", ["tiny", "l24"])
@pytest.mark.parametrize("tile", [None, "32", "64", "1288", "256", "64128"])
def test_split_matvec_bound(ctx, kind, tile, prec, monkeypatch):
    from paper_2407_07411_amd.heff import FP32, SPLIT_BF16X3
    print("case", kind, tile, prec, flush=True)
    if tile:
        monkeypatch.setenv("DMRG_HEFF_TILE", tile)
    prob = tiny_problem(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3) if kind == "tiny" else _l24(2)
    h = gpu_heff(ctx, prob, prec=SPLIT_BF16X3 if prec == "split" else FP32)
    y = h.apply(prob.psi.to("cuda")).cpu().numpy()
    ref = heff_apply(prob)
    err = rel(y, ref)
    print("split rel err", err, flush=True)
    assert err <= SPLIT_TOL
    assert err > 0.0  # the split kernels ran, not the FP64 ones


@pytest.mark.parametrize("prec", ["split", "fp32"])
def test_split_davidson_fp64_tail(ctx, prec):
    from paper_2407_07411_amd.heff import FP32, SPLIT_BF16X3, davidson
    prob = tiny_problem(seed=6, L=10, n_elec=10, D=24, pairs=3)
    e0 = np.linalg.eigvalsh(heff_dense(prob))[0]
    h = gpu_heff(ctx, prob, prec=SPLIT_BF16X3 if prec == "split" else FP32)
    psi = prob.psi.to("cuda").clone()
    res = davidson(h, psi, tol=1e-9, fp64_tail=60)
    print(res, e0, flush=True)
    assert res["converged"] and res["tail_iters"] >= 1
    assert abs(res["energy"] - e0) < 1e-8


@pytest.mark.parametrize("kind", ["tiny", "l24"])
@pytest.mark.parametrize("tile", [None, "32", "64", "64128"])
def test_presplit_operands_bit_identical(ctx, kind, tile, monkeypatch):
    """Split precision with the vector and the intermediates held pre-split
    (packed once by the kernels that produce them) equals the form that
    splits every operand while staging it, bit for bit: both make the same
    slices, so every product and every sum is the same.  Eager and graph
    replays, the graph twice with other work between."""
    from paper_2407_07411_amd.heff import SPLIT_BF16X3
    print("case", kind, tile, flush=True)
    if tile:
        monkeypatch.setenv("DMRG_HEFF_TILE", tile)
    prob = tiny_problem(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3) if kind == "tiny" else _l24(2)
    psi = prob.psi.to("cuda")
    monkeypatch.setenv("DMRG_HEFF_SPLIT_UNPACKED", "1")
    h0 = gpu_heff(ctx, prob, prec=SPLIT_BF16X3)
    ref = h0.apply(psi)
    monkeypatch.delenv("DMRG_HEFF_SPLIT_UNPACKED")
    h1 = gpu_heff(ctx, prob, prec=SPLIT_BF16X3)
    y = h1.apply(psi)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        h1.use_graph(True)
        out = torch.empty_like(psi)
        for _ in range(2):
            out.zero_()
            h1.apply(psi, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            h0.apply(psi * 0.5)  # other work between the replays
            torch.cuda.synchronize()
        h1.use_graph(False)


def test_fp64_accumulating_128_kernel_in_a_child_process():
    """The FP64-accumulating 128x128 split kernel (sixteen 32x32 waves,
    selected by DMRG_HEFF_SPLIT_ACC32=0, which the library reads once per
    process) on the L=24 problem with every product forced onto the
    128x128 shape, in a child process, under the stated bound."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import json, torch\n"
        "from oracle.heff import heff_apply\n"
        "from tests.test_gpu_heff import _l24, gpu_heff, rel\n"
        "from paper_2407_07411_amd.heff import Context, SPLIT_BF16X3\n"
        "prob = _l24(2)\n"
        "h = gpu_heff(Context(0), prob, prec=SPLIT_BF16X3)\n"
        "y = h.apply(prob.psi.to('cuda')).cpu().numpy()\n"
        "torch.cuda.synchronize()\n"
        "print(json.dumps({'err': rel(y, heff_apply(prob))}), flush=True)\n")
    env = dict(os.environ, DMRG_HEFF_SPLIT_ACC32="0", DMRG_HEFF_TILE="1288",
               PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    print("case split acc64 128x128 child process", flush=True)
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    err = json.loads(out.stdout.strip().splitlines()[-1])["err"]
    print("split acc64 rel err", err, flush=True)
    assert 0.0 < err <= SPLIT_TOL

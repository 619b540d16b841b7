"""Whole-size parity of the SU(2) form: the CAS(63,58)-shaped doublet bond at
D = 4096 multiplets with operator pools capped to 150 GB, as the benchmark
runs it; one matvec per precision in the benchmark's launch configuration.

The oracle computes sampled entries by the definition of the reduced matvec
(oracle.su2.heff_entries_blocks_su2, itself checked against the full oracle
on the CPU): the first and last row and column of every output block, plus
interior rows and columns of the
largest, a middle and the smallest block.  Each FP64 entry must agree to
1e-12 times the sum of the absolute values of its products; the split and
FP32-operand matvecs to their stated 1e-5 bound (norm-wise against FP64, and
entry-wise on the samples)."""
import gc

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

POOL_BYTES = int(150e9)
SPLIT_TOL = 1e-5


def _sample(n):
    return sorted({0, n - 1, n // 2, (n * 2) // 3})


@pytest.mark.timeout(600)
def test_su2_whole_size_sampled_entries():
    from oracle.su2 import heff_entries_blocks_su2, layout_su2
    from paper_2407_07411_amd import heff as H
    from synth.su2 import make_workload_su2

    dev = torch.device("cuda", 0)
    print("case su2_cas63_58_d4096", flush=True)
    prob = make_workload_su2("su2_cas63_58_d4096", device=dev, pool_budget_bytes=POOL_BYTES)
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    try:
        with torch.cuda.stream(stream):
            ctx = H.Context(0)
            h = H.HeffSU2(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                          prob.right_pool)
            outs = {}
            for lab, prec in (("fp64", H.FP64), ("split", H.SPLIT_BF16X3), ("fp32", H.FP32)):
                h.set_precision(prec)
                outs[lab] = h.apply(prob.psi)
            h.set_precision(H.FP64)
        torch.cuda.synchronize()
        y = outs["fp64"]
        for lab in ("split", "fp32"):
            err = float(torch.linalg.vector_norm(outs[lab] - y) / torch.linalg.vector_norm(y))
            print("su2", lab, "rel err", err, flush=True)
            assert 0.0 < err <= SPLIT_TOL
        ys = {k: v.cpu().numpy() for k, v in outs.items()}
        del h, ctx, outs
        lay = layout_su2(prob)
        order = sorted(lay.blocks, key=lambda b: int(lay.Ld[b[0]]) * int(lay.Rd[b[1]]))
        samples = {}
        for b in lay.blocks:
            nr, nc = int(lay.Ld[b[0]]), int(lay.Rd[b[1]])
            samples[b] = (sorted({0, nr - 1}), sorted({0, nc - 1}))
        for b in (order[-1], order[len(order) // 2], order[0]):
            samples[b] = (_sample(int(lay.Ld[b[0]])), _sample(int(lay.Rd[b[1]])))
        import time
        print("sampling", len(samples), "output blocks", flush=True)
        t0 = time.time()
        got = heff_entries_blocks_su2(prob, samples)
        print("oracle seconds", round(time.time() - t0, 1), flush=True)
        worst = 0.0
        for b, (rows, cols) in samples.items():
            val, mag = got[b]
            ent = lay.block(ys["fp64"], *b)[np.ix_(rows, cols)]
            err = np.abs(ent - val)
            worst = max(worst, float((err / (mag + 1e-300)).max()))
            assert np.all(err <= 1e-12 * mag + 1e-300), (b, err.max(), mag.max())
            for lab in ("split", "fp32"):
                ent_r = lay.block(ys[lab], *b)[np.ix_(rows, cols)]
                assert np.all(np.abs(ent_r - val) <= SPLIT_TOL * mag + 1e-300), (lab, b)
        print("su2 worst FP64 entry error / product scale", worst, flush=True)
    finally:
        del prob
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

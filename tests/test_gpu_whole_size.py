"""Whole-size parity: the two benchmark-sized workloads (CAS(63,58)-shaped at
D=4096 and CAS(113,76)-shaped at D=8192, operator pools capped to 150 GB as in
the benchmark), one matvec in the benchmark's launch configuration (default
tile rule and workspace), checked on sampled entries against the oracle.

A whole output block is out of the oracle's reach at these sizes, so the
oracle computes single entries by the same definition: the first and last
row and column of EVERY output block (so every block's sum, its K-cut parts
and its edge tiles are looked at), plus interior rows and columns of the
largest, a middle and the smallest block.  Each
entry must agree to 1e-12 times the sum of the absolute values of the
products that enter it (the scale of its FP64 rounding error).  The split
and FP32-operand matvecs are checked against the FP64 one norm-wise (their
stated 1e-5 bound) and on the same sampled entries."""
import gc

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

POOL_BYTES = int(150e9)
SPLIT_TOL = 1e-5


def _sample(n, k=3):
    idx = sorted({0, n - 1, n // 2, (n * 2) // 3})
    return idx[:k + 1]


@pytest.mark.parametrize("name", ["cas63_58_d4096", "cas113_76_d8192"])
def test_whole_size_sampled_entries(name):
    from oracle.heff import heff_entries_blocks, layout_of
    from paper_2407_07411_amd import heff as H
    from synth.problem import WORKLOADS, make_problem

    w = WORKLOADS[name]
    dev = torch.device("cuda", 0)
    print("case", name, flush=True)
    prob = make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], device=dev,
                        pool_budget_bytes=POOL_BYTES)
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    try:
        with torch.cuda.stream(stream):
            ctx = H.Context(0)
            h = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                       prob.right_pool)
            y = torch.empty_like(prob.psi)
            h.apply(prob.psi, y)
            ys = torch.empty_like(prob.psi)
            h.set_precision(H.SPLIT_BF16X3)
            h.apply(prob.psi, ys)
            yf = torch.empty_like(prob.psi)
            h.set_precision(H.FP32)
            h.apply(prob.psi, yf)
            h.set_precision(H.FP64)
        torch.cuda.synchronize()
        for lab, yr in (("split", ys), ("fp32", yf)):
            err = float(torch.linalg.vector_norm(yr - y) / torch.linalg.vector_norm(y))
            print(name, lab, "rel err", err, flush=True)
            assert 0.0 < err <= SPLIT_TOL
        y64 = y.cpu().numpy()
        y16 = ys.cpu().numpy()
        y32 = yf.cpu().numpy()
        del h, ctx
        lay = layout_of(prob)
        order = sorted(lay.partner, key=lambda a: int(lay.Ld[a]) * int(lay.Rd[lay.partner[a]]))
        samples = {}
        for b in lay.partner:
            nr, nc = int(lay.Ld[b]), int(lay.Rd[lay.partner[b]])
            samples[b] = (sorted({0, nr - 1}), sorted({0, nc - 1}))
        for b in (order[-1], order[len(order) // 2], order[0]):
            nr, nc = int(lay.Ld[b]), int(lay.Rd[lay.partner[b]])
            samples[b] = (_sample(nr), _sample(nc))
        print(name, "sampling", len(samples), "output blocks", flush=True)
        got = heff_entries_blocks(prob, samples)
        worst = 0.0
        for b, (rows, cols) in samples.items():
            val, mag = got[b]
            ent = lay.block(y64, b)[np.ix_(rows, cols)]
            err = np.abs(ent - val)
            worst = max(worst, float((err / (mag + 1e-300)).max()))
            assert np.all(err <= 1e-12 * mag + 1e-300), (b, err.max(), mag.max())
            for yr in (y16, y32):
                ent_r = lay.block(yr, b)[np.ix_(rows, cols)]
                assert np.all(np.abs(ent_r - val) <= SPLIT_TOL * mag + 1e-300), b
        print(name, "worst FP64 entry error / product scale", worst, flush=True)
    finally:
        del prob
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def test_d8192_graph_davidson_fp64_and_split():
    """CAS(113,76)-shaped sectors at D=8192 (pools capped to 20 GB: fewer
    operator pairs, the same block shapes), Davidson to a 1e-6 residual with
    hipGraph-captured iterations: FP64, and split precision with an FP64 tail.
    The two energies agree to 1e-8."""
    from paper_2407_07411_amd import heff as H
    from synth.problem import WORKLOADS, make_problem

    w = WORKLOADS["cas113_76_d8192"]
    dev = torch.device("cuda", 0)
    prob = make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], device=dev,
                        pool_budget_bytes=int(20e9))
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    try:
        with torch.cuda.stream(stream):
            ctx = H.Context(0)
            h = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                       prob.right_pool)
            out = {}
            for label, prec, tail in (("fp64", H.FP64, 0), ("split", H.SPLIT_BF16X3, 40),
                                      ("fp32", H.FP32, 40)):
                h.set_precision(prec)
                psi = prob.psi.clone()
                out[label] = H.davidson(h, psi, tol=1e-6, max_iter=80, use_graph=True, fp64_tail=tail,
                                        start_from_diag=True)
                print(label, out[label], flush=True)
            h.set_precision(H.FP64)
        torch.cuda.synchronize()
        for lab in ("split", "fp32"):
            assert out["fp64"]["converged"] and out[lab]["converged"]
            assert out[lab]["split_iters"] >= 1
            assert abs(out["fp64"]["energy"] - out[lab]["energy"]) < 1e-8
        del h, ctx
    finally:
        del prob
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

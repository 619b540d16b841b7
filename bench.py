"""Benchmark: two-site H_eff . psi inside Davidson on one MI355X.

Workload (default): the CAS(63,58)-shaped synthetic middle bond at D=4096
(58 orbitals, 63 electrons, 2Sz=1; enlarged sectors of 1..834 rows), operator
pools capped uniformly in term count to --pool-gb.  A step is one Davidson
iteration (Rayleigh-Ritz, residual, preconditioner, Gram-Schmidt and one
H_eff matvec), all on the device in FP64, its stages replayed from hipGraphs.
`value` is the algorithmic FP64
FLOP rate of the matvecs over the timed steps (wall clock of whole steps).

Also reported: the matvec alone (FP64, split BF16x3, FP32 operands), the roofline of the
dominant kernel from per-launch HIP events, Davidson to a 1e-6 residual with
hipGraph-captured iterations (FP64, and split or FP32 operands with an FP64
tail), and the CPU FP64 oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--pool-gb G]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "gemm_f64_kernel<32,32,16,1,1>", 1: "gemm_f64_kernel<64,64,16,2,2>",
                2: "gemm_f64_kernel<128,128,16,2,2>", 3: "gemm_f64_kernel<128,128,16,4,2>",
                4: "gemm_f64_kernel<256,128,16,4,2>", 5: "gemm_f64_kernel<64,128,16,2,4>",
                16: "gemm_split_kernel<32,32,1,1>",
                17: "gemm_split_kernel<64,64,2,2>", 18: "gemm_split_kernel<128,128,2,2>",
                19: "gemm_split_kernel<128,128,4,4,1,64>", 20: "gemm_split_kernel<256,128,4,4>",
                21: "gemm_split_kernel<64,128,2,4>",
                6: "gemm_f64_dma_kernel<64,128,2,4,2>", 7: "gemm_f64_dma_kernel<64,128,2,4,3>",
                8: "gemm_f64_dma_kernel<128,128,4,2,2>", 9: "gemm_f64_dma_kernel<64,64,2,2,2>",
                10: "gemm_f64_dma_kernel<32,32,1,1,2>",
                32: "reduce_kernel", 64: "persist_f64_kernel",
                48: "gemm_f32_kernel<32,32,32,1,1>", 49: "gemm_f32_kernel<64,64,32,2,2>",
                50: "gemm_f32_kernel<128,128,16,2,2>", 51: "gemm_f32_kernel<128,128,32,4,2>",
                52: "gemm_f32_kernel<256,128,16,4,2>", 53: "gemm_f32_kernel<64,128,32,2,4>"}


ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_SOURCES = ("paper_2407_07411_amd/csrc", "include", "synth")


def sources_digest():
    """SHA-256 over the kernel, plan and input-generator sources: a stored HBM
    byte count is reported only while these are unchanged."""
    import hashlib
    hsh = hashlib.sha256()
    for d in TRAFFIC_SOURCES:
        for name in sorted(os.listdir(os.path.join(ROOT, d))):
            if name.endswith((".hip", ".h", ".py")):
                hsh.update(name.encode())
                with open(os.path.join(ROOT, d, name), "rb") as f:
                    hsh.update(f.read())
    return hsh.hexdigest()


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or
    None when there is none or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    digest, val = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("sources_sha256:"):
                digest = line.split(":", 1)[1].strip()
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 2 and cells[0].strip("`").replace(" ", "") == kernel.replace(" ", ""):
                try:
                    val = float(cells[-1])
                except ValueError:
                    pass
    return val if digest == sources_digest() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cas63_58_d4096")
    ap.add_argument("--pool-gb", type=float, default=150.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the Davidson-to-tolerance runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (tile shapes per size class, per-phase or persistent launch)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the off-path measurements (SVD truncation, out-of-core matvec, adjoint at L=24, sweeps)")
    ap.add_argument("--only-out-of-core", action="store_true",
                    help="run only the out-of-core matvec measurement and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device twice, by the runtime's copy and by an "
                         "elementwise kernel (reference dispatches for HBM byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the term-sharded "
              "multi-GPU layout is described in the design notes, not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2407_07411_amd import heff as H
    from synth.problem import WORKLOADS, make_problem

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only_out_of_core:
        print(json.dumps(dict(workload=args.workload, out_of_core=streamed_timing(dev, w))), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # the runtime's device-to-device copy
        torch.neg(src, out=dst)  # a plain elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        log("copied 1 GiB twice (counter calibration)")
    t0 = time.time()
    prob = make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], device=dev,
                        pool_budget_bytes=int(args.pool_gb * 1e9))
    torch.cuda.synchronize()
    log(f"generated {args.workload}: {prob.meta['n_terms']} terms, pools {prob.meta['pool_bytes']/1e9:.1f} GB, "
        f"psi {prob.meta['psi_len']} ({time.time()-t0:.1f} s)")
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(stream):
        ctx = H.Context(0)
        t0 = time.time()
        h = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                   prob.right_pool)
        flops, alg_bytes = h.flops()
        plan_s = time.time() - t0
        log(f"plan: {flops/1e12:.2f} TFLOP/matvec, workspace {h.workspace_bytes()/1e9:.2f} GB "
            f"({plan_s:.1f} s)")
        x = prob.psi.clone()
        y = torch.empty_like(x)
        # the two launch forms of the FP64 matvec (bit-identical results)
        forms = {}
        for pers in (False, True):
            h.set_persistent(pers)
            h.apply(x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(2):
                h.apply(x, y)
            e1.record(stream)
            torch.cuda.synchronize()
            forms["persistent" if pers else "per_phase"] = e0.elapsed_time(e1) / 2
        h.check()
        h.set_persistent(False)
        log(f"untuned matvec: per-phase launches {forms['per_phase']:.1f} ms, one persistent launch "
            f"{forms['persistent']:.1f} ms")
        tune_s = None
        if not args.no_tune:
            t0 = time.time()
            h.autotune(x, y, reps=2)
            tune_s = time.time() - t0
            log(f"autotuned ({tune_s:.1f} s)")
        kid0, _ = h.launches()
        form = "persistent" if len(kid0) == 1 and int(kid0[0]) == 64 else "per_phase"
        log(f"matvec form: {form}")
        # marker for kernel traces: the dispatches between this spin kernel
        # and the next are the kept plan's matvecs and Davidson iterations
        # (the tuner before it launches the same kernels on subsets)
        torch.cuda._sleep(1000)

        # ---- matvec alone (FP64): warm-up, then HIP events on this stream
        for _ in range(2):
            h.apply(x, y)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 3
        ev[0].record(stream)
        for _ in range(reps):
            h.apply(x, y)
        ev[1].record(stream)
        torch.cuda.synchronize()
        mv_ms = ev[0].elapsed_time(ev[1]) / reps
        log(f"matvec fp64 {mv_ms:.2f} ms -> {flops/mv_ms/1e9:.2f} TFLOPS")

        # ---- roofline of the dominant kernel from per-launch events
        kid, kflops = h.launches()
        ms = h.apply_profiled(x, y)
        per = {}
        for k, f, m in zip(kid.tolist(), kflops.tolist(), ms.tolist()):
            a = per.setdefault(int(k), [0.0, 0.0, 0])
            a[0] += f
            a[1] += m
            a[2] += 1
        for k in sorted(per):
            f_, m_, n_ = per[k]
            log(f"  {KERNEL_NAMES.get(k, k)}: {n_} launches, {m_:.1f} ms ({100*m_/float(ms.sum()):.0f}%), "
                f"{f_/(m_/1e3)/1e12 if m_ > 0 else 0:.1f} TFLOP/s")
        dom = max(per, key=lambda k: per[k][1])
        dflops, dms, dn = per[dom]
        achieved = dflops / (dms / 1e3) / 1e12
        dname = KERNEL_NAMES.get(dom, str(dom))
        traffic = profiled_traffic(dname, args.workload) if args.pool_gb == 150.0 else None
        roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=traffic,
                        traffic_unit="bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                        traffic_source="read from the committed counter summary of this workload while the "
                                       "kernel, plan and generator sources match its SHA-256 (else null); "
                                       "not counted in this run",
                        kernel=dname, launches=dn,
                        avg_launch_ms=round(dms / dn, 4), flops_per_launch=dflops / dn,
                        share_of_matvec=round(dms / float(ms.sum()), 3))
        log(f"dominant kernel {roofline['kernel']}: {achieved:.2f} TFLOP/s over {dn} launches")

        # ---- timed Davidson iterations (the step)
        import ctypes

        from paper_2407_07411_amd import _lib
        L = _lib.lib()
        # hipGraph-captured iteration stages
        opts = _lib.DavOpts(args.warmup + args.steps + 8, 24, 2, 1, 0.0, 0, 0)
        d = ctypes.c_void_p()
        ctx.sync_stream()
        _lib.check(L.dmrg_davidson_create(h.h, ctypes.byref(opts), ctypes.c_void_p(x.data_ptr()), ctypes.byref(d)))
        res = _lib.DavResult()
        for _ in range(args.warmup):
            _lib.check(L.dmrg_davidson_step(d, ctypes.byref(res)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _lib.check(L.dmrg_davidson_step(d, ctypes.byref(res)))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        L.dmrg_davidson_destroy(d)
        step_ms = el / args.steps * 1e3
        value = flops * args.steps / el / 1e12
        log(f"davidson step {step_ms:.2f} ms -> {value:.2f} TFLOPS (residual {res.residual:.3e})")

        # ---- diagonal (the preconditioner; once per bond)
        dg = torch.empty_like(x)
        h.diag(dg)
        ev[0].record(stream)
        h.diag(dg)
        ev[1].record(stream)
        torch.cuda.synchronize()
        diag_ms = ev[0].elapsed_time(ev[1])
        extra = dict(plan_seconds=round(plan_s, 3), tune_seconds=None if tune_s is None else round(tune_s, 3),
                     matvec_form=form, untuned_matvec_ms=dict((k, round(v, 3)) for k, v in forms.items()),
                     diag_ms=round(diag_ms, 3),
                     matvec_ms_fp64=round(mv_ms, 3), matvec_tflops_fp64=round(flops / mv_ms / 1e9, 3),
                     davidson_iter_ms_fp64=round(step_ms, 3), alg_tflop_per_matvec=round(flops / 1e12, 4),
                     alg_intensity_flop_per_byte=round(flops / alg_bytes, 1))

        # ---- split precision: matvec rate and error against the FP64 matvec
        y64 = y.clone()
        h.set_precision(H.SPLIT_BF16X3)
        h.apply(x, y)
        ev[0].record(stream)
        for _ in range(reps):
            h.apply(x, y)
        ev[1].record(stream)
        torch.cuda.synchronize()
        sp_ms = ev[0].elapsed_time(ev[1]) / reps
        sp_err = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
        extra.update(matvec_ms_split=round(sp_ms, 3), matvec_tflops_split=round(flops / sp_ms / 1e9, 3),
                     split_speedup=round(mv_ms / sp_ms, 3), split_matvec_rel_err=sp_err)
        log(f"matvec split {sp_ms:.2f} ms -> {flops/sp_ms/1e9:.2f} TFLOPS (FP64-equivalent), rel err {sp_err:.2e}")

        # ---- FP32 operands on the FP32 matrix cores: matvec rate and error
        h.set_precision(H.FP32)
        h.apply(x, y)
        ev[0].record(stream)
        for _ in range(reps):
            h.apply(x, y)
        ev[1].record(stream)
        torch.cuda.synchronize()
        f32_ms = ev[0].elapsed_time(ev[1]) / reps
        f32_err = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
        h.set_precision(H.FP64)
        extra.update(matvec_ms_fp32=round(f32_ms, 3), matvec_tflops_fp32=round(flops / f32_ms / 1e9, 3),
                     fp32_speedup=round(mv_ms / f32_ms, 3), fp32_matvec_rel_err=f32_err)
        log(f"matvec fp32 {f32_ms:.2f} ms -> {flops/f32_ms/1e9:.2f} TFLOPS (FP64-equivalent), rel err {f32_err:.2e}")
        torch.cuda._sleep(1000)  # end marker of the measured matvecs for kernel traces

        # ---- Davidson to the 1e-6 residual from the lowest diagonal element
        ground = None
        if not args.no_solve:
            for label, prec, tail in (("fp64", H.FP64, 0), ("split_fp64_tail", H.SPLIT_BF16X3, 40),
                                      ("fp32_fp64_tail", H.FP32, 40)):
                h.set_precision(prec)
                psi = prob.psi.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = H.davidson(h, psi, tol=1e-6, max_iter=60, fp64_tail=tail, start_from_diag=True,
                               use_graph=True)
                torch.cuda.synchronize()
                r["seconds"] = round(time.perf_counter() - t0, 3)
                extra["davidson_" + label] = r
                if label == "fp64":
                    ground = psi
                log(f"davidson {label}:", r)
            h.set_precision(H.FP64)
            for lab in ("split", "fp32"):
                r = extra[f"davidson_{lab}_fp64_tail"]
                if extra["davidson_fp64"]["converged"] and r["converged"]:
                    e64 = extra["davidson_fp64"]["energy"]
                    extra[f"{lab}_energy_error"] = abs(e64 - r["energy"])
                    # the reduced-precision phase alone, before the FP64 tail
                    extra[f"{lab}_only_energy_error"] = abs(e64 - r["split_energy"])
                    extra[f"{lab}_only_residual"] = r["split_residual"]
                    extra[f"{lab}_solve_speedup"] = round(extra["davidson_fp64"]["seconds"] / r["seconds"], 3)

        # ---- off the timed path, measured: SVD truncation of the FP64 ground state
        if not args.no_extra:
            torch.cuda.synchronize()
            psi = ground if ground is not None else prob.psi
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                kept, U, S, Vt, terr = H.svd_truncate(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, psi,
                                                      max_keep=w["D"])
                torch.cuda.synchronize()
                svd_s = time.perf_counter() - t0
            extra["svd_truncate"] = dict(seconds=round(svd_s, 3), kept=int(np.sum(kept)), max_keep=w["D"],
                                         trunc_err=terr,
                                         state="FP64 ground state" if ground is not None else "random psi")
            log(f"svd truncation: {svd_s:.3f} s, kept {int(np.sum(kept))}, error {terr:.3e}")
            del U, S, Vt
    cpu = None
    if not args.no_cpu:
        lid = {tuple(q): i for i, q in enumerate(np.asarray(prob.Lq).tolist())}
        rid = {tuple(q): i for i, q in enumerate(np.asarray(prob.Rq).tolist())}
        try:
            cpu = cpu_baseline(prob, args.cpu_seconds, lid, rid)
        except Exception as e:  # the GPU result stands without it
            log("cpu baseline failed:", repr(e))
    pmeta = dict(prob.meta)
    if not args.no_extra:
        # the off-path legs need the memory of this workload's plan and pools
        del h, x, y, prob
        torch.cuda.empty_cache()
        extra["out_of_core_" + args.workload] = streamed_timing(dev, w)
        extra["su2_cas63_58_d4096"] = su2_timing(dev)
        extra["adjoint_l24_d1024"] = adjoint_timing(dev)
        # the L=24, D=1024 single FP64 matvec with all 1226 terms, on its own
        extra["matvec_tflops_l24_d1024_all_terms"] = extra["adjoint_l24_d1024"]["forward_tflops"]
        extra["matvec_tflops_l24_d1024_all_terms_tuned"] = extra["adjoint_l24_d1024"]["forward_tflops_tuned"]
        extra["sweeps_l8_d64"] = sweep_timing()
    out = dict(metric="H_eff\u00b7\u03c8 TFLOPS/GPU (FP64 vs split-prec) at D=4096; Davidson iter time",
               value=round(value, 3),
               unit="TFLOPS", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(step_ms, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=args.workload, L=w["L"], n_elec=w["n_elec"], two_sz=w["two_sz"], D=w["D"],
                           terms=pmeta["n_terms"], stored_pairs=pmeta["n_pairs"],
                           pool_gb=round(pmeta["pool_bytes"] / 1e9, 2), psi_len=pmeta["psi_len"],
                           step="one Davidson iteration incl. one H_eff matvec, hipGraph-captured stages"),
               roofline=roofline, cpu_baseline=cpu, **extra)
    print(json.dumps(out), flush=True)


def adjoint_timing(dev):
    """Forward matvec and hand-written adjoint (psi-bar and both operator-pool
    gradients, intermediates recomputed) on the L=24, D=1024 workload with
    every operator pair, timed with HIP events on the library's stream."""
    import torch

    from paper_2407_07411_amd import heff as H
    from synth.problem import WORKLOADS, make_problem
    w = WORKLOADS["l24_d1024"]
    prob = make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], device=dev)
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(stream):
        ctx = H.Context(0)
        h = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                   prob.right_pool)
        flops, _ = h.flops()
        x = prob.psi.clone()
        y = torch.empty_like(x)
        yb = torch.randn(x.numel(), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(3))
        pb = torch.zeros_like(x)
        lb = torch.zeros_like(prob.left_pool)
        rb = torch.zeros_like(prob.right_pool)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for rep in range(2):  # the first pass builds the adjoint plan
            ev[0].record(stream)
            h.apply(x, y)
            ev[1].record(stream)
            h.adjoint(x, yb, pb, lb, rb)
            ev[2].record(stream)
        torch.cuda.synchronize()
        fwd_ms = ev[0].elapsed_time(ev[1])
        adj_ms = ev[1].elapsed_time(ev[2])
        # the forward with the plan autotuned (tile shapes and launch form)
        h.autotune(x, y, reps=3)
        h.apply(x, y)
        ev[0].record(stream)
        for _ in range(5):
            h.apply(x, y)
        ev[1].record(stream)
        torch.cuda.synchronize()
        tuned_ms = ev[0].elapsed_time(ev[1]) / 5
    out = dict(terms=prob.meta["n_terms"], forward_ms=round(fwd_ms, 3),
               forward_tflops=round(flops / fwd_ms / 1e9, 3), forward_ms_tuned=round(tuned_ms, 3),
               forward_tflops_tuned=round(flops / tuned_ms / 1e9, 3), adjoint_ms=round(adj_ms, 3),
               adjoint_over_forward=round(adj_ms / fwd_ms, 3),
               adjoint_outputs="psi-bar, left-pool and right-pool gradients")
    log("adjoint l24_d1024:", out)
    return out


def streamed_timing(dev, w, pool_gb=24.0):
    """The out-of-core form on the same workload with pools capped to
    pool_gb: the pools in pinned host memory, a device budget of 75% of them
    (the blocks that fit copied once, the rest streamed through two slots
    per matvec) and a budget of 8 GB with nothing resident.  Each matvec is
    timed with HIP events and compared with the plan over device pools; the
    bound is the larger of that plan's time and the streamed bytes at the
    measured pinned host-to-device rate."""
    import os

    import torch

    from paper_2407_07411_amd import heff as H
    from synth.problem import make_problem
    prob = make_problem(w["L"], w["n_elec"], w["two_sz"], w["D"], w["seed"], device=dev,
                        pool_budget_bytes=int(pool_gb * 1e9))
    pb = prob.meta["pool_bytes"]
    lp = torch.empty(prob.left_pool.numel(), dtype=torch.float64, pin_memory=True)
    rp = torch.empty(prob.right_pool.numel(), dtype=torch.float64, pin_memory=True)
    lp.copy_(prob.left_pool)
    rp.copy_(prob.right_pool)
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps=3):
        fn()
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    out = dict(pool_gb=round(pb / 1e9, 3), terms=prob.meta["n_terms"])
    with torch.cuda.stream(stream):
        n = min(lp.numel(), 1 << 29)
        dst = torch.empty(n, dtype=torch.float64, device=dev)
        h2d_ms = timed(lambda: dst.copy_(lp[:n], non_blocking=True))
        h2d = n * 8 / h2d_ms / 1e6
        del dst
        ctx = H.Context(0)
        x = prob.psi.clone()
        h = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool, prob.right_pool)
        flops, _ = h.flops()
        y_ref = h.apply(x)
        dev_ms = timed(lambda: h.apply(x, y_ref))
        del h
        prob.left_pool = prob.right_pool = None
        torch.cuda.empty_cache()
        out.update(h2d_gbps=round(h2d, 2), device_pools_matvec_ms=round(dev_ms, 3),
                   device_pools_tflops=round(flops / dev_ms / 1e9, 3))
        for label, dbytes, resident_kb in (("budget_75pct", int(0.75 * pb), None), ("budget_8gb_all_streamed",
                                                                                     int(8e9), "0")):
            if resident_kb is None:
                os.environ.pop("DMRG_HEFF_STREAM_RESIDENT_KB", None)
            else:
                os.environ["DMRG_HEFF_STREAM_RESIDENT_KB"] = resident_kb
            hs = H.Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, lp, rp, device_bytes=dbytes)
            os.environ.pop("DMRG_HEFF_STREAM_RESIDENT_KB", None)
            rb, sb, rw, sw = hs.stream_info()
            y = torch.empty_like(x)
            ms = timed(lambda: hs.apply(x, y))
            err = float(torch.linalg.vector_norm(y - y_ref) / torch.linalg.vector_norm(y_ref))
            bound = max(dev_ms, sb / h2d / 1e6)
            out[label] = dict(device_gb=round(dbytes / 1e9, 3), resident_gb=round(rb / 1e9, 3),
                              streamed_gb_per_matvec=round(sb / 1e9, 3), resident_waves=rw, streamed_waves=sw,
                              matvec_ms=round(ms, 3), pcie_inclusive_tflops=round(flops / ms / 1e9, 3),
                              bound_ms=round(bound, 3), frac_of_bound=round(bound / ms, 4),
                              rel_err_vs_device_pools=err)
            del hs
    log("out-of-core:", out)
    return out


def su2_timing(dev, pool_gb=150.0):
    """The SU(2) spin-adapted form at the paper's own bond dimension: the
    CAS(63,58)-shaped doublet bond with D = 4096 multiplets per block,
    operator pairs capped uniformly to pool_gb; FP64, split and FP32-operand
    matvecs timed with HIP events, reduced precisions compared with FP64."""
    import torch

    from paper_2407_07411_amd import heff as H
    from synth.su2 import WORKLOADS_SU2, make_workload_su2
    name = "su2_cas63_58_d4096"
    prob = make_workload_su2(name, device=dev, pool_budget_bytes=int(pool_gb * 1e9))
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = dict(D_multiplets=WORKLOADS_SU2[name]["D"], two_s=WORKLOADS_SU2[name]["two_s"],
               terms=prob.meta["n_terms"], pool_gb=round(prob.meta["pool_bytes"] / 1e9, 2),
               psi_len=prob.meta["psi_len"], max_sector_multiplets=int(max(prob.Ld.max(), prob.Rd.max())))
    with torch.cuda.stream(stream):
        ctx = H.Context(0)
        t0 = time.time()
        h = H.HeffSU2(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool,
                      prob.right_pool)
        flops, _ = h.flops()
        out.update(plan_seconds=round(time.time() - t0, 3), alg_tflop_per_matvec=round(flops / 1e12, 3))
        x = prob.psi.clone()
        y64 = torch.empty_like(x)
        y = torch.empty_like(x)
        for prec, lab in ((H.FP64, "fp64"), (H.SPLIT_BF16X3, "split"), (H.FP32, "fp32")):
            h.set_precision(prec)
            tgt = y64 if lab == "fp64" else y
            h.apply(x, tgt)
            ev[0].record(stream)
            for _ in range(3):
                h.apply(x, tgt)
            ev[1].record(stream)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 3
            out[f"matvec_ms_{lab}"] = round(ms, 3)
            out[f"matvec_tflops_{lab}"] = round(flops / ms / 1e9, 3)
            if lab != "fp64":
                out[f"{lab}_rel_err"] = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
        h.set_precision(H.FP64)
        # Davidson iterations (one hipGraph and one matvec each), as the main step
        import ctypes

        from paper_2407_07411_amd import _lib
        L = _lib.lib()
        opts = _lib.DavOpts(8, 24, 2, 1, 0.0, 0, 1)
        d = ctypes.c_void_p()
        ctx.sync_stream()
        _lib.check(L.dmrg_davidson_create(h.h, ctypes.byref(opts), None, ctypes.byref(d)))
        res = _lib.DavResult()
        for _ in range(2):
            _lib.check(L.dmrg_davidson_step(d, ctypes.byref(res)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            _lib.check(L.dmrg_davidson_step(d, ctypes.byref(res)))
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) / 2 * 1e3
        L.dmrg_davidson_destroy(d)
        out.update(davidson_iter_ms_fp64=round(step_ms, 3), davidson_iter_tflops_fp64=round(flops / step_ms / 1e9, 3))
    out["split_speedup"] = round(out["matvec_ms_fp64"] / out["matvec_ms_split"], 3)
    del h, prob
    torch.cuda.empty_cache()
    log("su2 cas63_58 D=4096 multiplets:", out)
    return out


def sweep_timing():
    """Two full two-site sweeps (left to right and back, twice) of the L=8,
    8-electron, Sz=0 chain at D=64: operator blocks built and renormalised by
    the library, Davidson to 1e-9 and SVD truncation at every step.  Reports
    the wall time and the lowest energy; its agreement with FCI is a GPU test,
    not measured here."""
    import torch

    from paper_2407_07411_amd.chain import Chain
    from paper_2407_07411_amd.heff import Context
    from synth.integrals import integrals
    h1, V = integrals(8, 1001)
    ctx = Context(0)
    ch = Chain(ctx, h1, V, 8, 0, D=64, seed=7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(2):
        steps += ch.sweep(+1, tol=1e-9)
        steps += ch.sweep(-1, tol=1e-9)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = dict(steps=len(steps), seconds=round(el, 3), ms_per_step=round(el / len(steps) * 1e3, 2),
               lowest_energy=min(s["energy"] for s in steps),
               converged=all(bool(s["converged"]) for s in steps))
    log("sweeps l8_d64:", out)
    return out


def cpu_baseline(prob, target_s, lid, rid):
    """The CPU FP64 oracle on a bounded sample: whole operator pairs (one
    term and its hermitian-conjugate partner) over every wavefunction block,
    drawn in a seeded random order until target_s seconds of CPU work."""
    terms = []
    for t in prob.terms:
        if t.one_sided:
            continue
        ol = {a: lid.get((q[0] + t.dq[0], q[1] + t.dq[1])) for a, q in enumerate(np.asarray(prob.Lq).tolist())}
        orr = {c: rid.get((r[0] - t.dq[0], r[1] - t.dq[1])) for c, r in enumerate(np.asarray(prob.Rq).tolist())}
        terms.append((t, ol, orr))
    return _cpu_sample(prob, terms, target_s)


def _cpu_sample(prob, terms, target_s):
    from oracle.heff import count_flops, heff_apply
    from synth.problem import Problem, Term
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    rng = np.random.default_rng(0)
    order = rng.permutation(len(terms))
    psi = prob.psi.cpu()
    flops = secs = 0.0
    n = 0
    for idx in order:
        t, ol, orr = terms[idx]
        lspan = [(int(o), int(o) + int(prob.Ld[ol[a]]) * int(prob.Ld[a])) for a, o in enumerate(t.left_off) if o >= 0]
        rspan = [(int(o), int(o) + int(prob.Rd[orr[c]]) * int(prob.Rd[c])) for c, o in enumerate(t.right_off) if o >= 0]
        l0, l1 = min(s for s, _ in lspan), max(e for _, e in lspan)
        r0, r1 = min(s for s, _ in rspan), max(e for _, e in rspan)
        lp = prob.left_pool[l0:l1].cpu()
        rp = prob.right_pool[r0:r1].cpu()
        tt = Term(dq=t.dq, odd=t.odd, hc=t.hc, one_sided=0, coeff=t.coeff,
                  left_off=np.where(t.left_off >= 0, t.left_off - l0, -1),
                  right_off=np.where(t.right_off >= 0, t.right_off - r0, -1))
        sub = Problem(prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, [tt], lp, rp, psi)
        t0 = time.perf_counter()
        heff_apply(sub)
        secs += time.perf_counter() - t0
        flops += count_flops(sub)
        n += 1
        if secs >= target_s:
            break
    n_terms = sum(1 + t.hc for t in prob.terms)
    return dict(value=round(flops / secs / 1e12, 5), unit="TFLOPS", cores=int(cores), kind="oracle",
                cpu_model=_cpu_model(), blas=_blas_vendor(),
                sample=f"{n} operator pairs (with their hc partners) of {n_terms} terms, full sector shapes, "
                       f"numpy float64 matvec, {secs:.1f} s")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _blas_vendor():
    try:
        from threadpoolctl import threadpool_info
        libs = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if libs:
            i = libs[0]
            return f"{i.get('internal_api')} {i.get('version')} ({i.get('threading_layer')}, " \
                   f"{i.get('num_threads')} threads)"
    except Exception:  # pragma: no cover
        pass
    return "unknown"


if __name__ == "__main__":
    main()

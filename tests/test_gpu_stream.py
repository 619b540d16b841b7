"""Out-of-core operators: the pools in pinned host memory, the blocks that fit
a device budget copied once, the rest copied through two staging slots on
a copy stream during every matvec.

* Everything resident (a budget above the pools), or everything streamed
  through slots larger than any workspace wave (resident part forced to
  zero): the waves and their order equal those of the plan over device
  pools, so every output element is summed in the same order and the
  results agree bit for bit, in every precision, on several consecutive
  applies (slots reused across calls) and for the diagonal.
* Mixed: a small resident part and slots of one pair's blocks, so resident
  and streamed waves interleave and slots alternate many times per apply:
  held to the oracle at 1e-12 (the FP64 matvec bound) and to the
  device-pool plan at 1e-12; Davidson converges to the same energy.
* Refusals: pageable or device pools, budgets below two slots, and the
  calls this form does not support."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.heff import heff_apply
from tests.conftest import tiny_problem, with_one_sided_hc
from tests.test_gpu_heff import _l24, rel

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": lambda: tiny_problem(seed=2, D=8, pairs=3),
    "tiny_hc": lambda: with_one_sided_hc(tiny_problem(seed=4, L=10, n_elec=9, two_sz=1, D=24, pairs=3), seed=4),
    "l24": lambda: _l24(2),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_07411_amd.heff import Context
    return Context(0)


def pinned(t):
    out = torch.empty(t.numel(), dtype=torch.float64, pin_memory=True)
    out.copy_(t.reshape(-1))
    return out


def device_plan(ctx, prob, prec=0):
    from paper_2407_07411_amd.heff import Heff
    return Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, prob.left_pool.to("cuda"),
                prob.right_pool.to("cuda"), prec=prec)


def streamed_plan(ctx, prob, device_bytes, prec=0):
    from paper_2407_07411_amd.heff import Heff
    return Heff(ctx, prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q, prob.terms, pinned(prob.left_pool),
                pinned(prob.right_pool), prec=prec, device_bytes=device_bytes)


def pool_bytes(prob):
    return 8 * (prob.left_pool.numel() + prob.right_pool.numel())


def inputs(prob, n=3):
    g = torch.Generator().manual_seed(11)
    xs = [prob.psi.to("cuda")]
    xs += [torch.randn(prob.psi.numel(), generator=g, dtype=torch.float64).to("cuda") for _ in range(n - 1)]
    return xs


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("mode", ["resident", "all_streamed"])
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_same_waves_bit_identical(ctx, name, mode, prec, monkeypatch):
    print("case stream", name, mode, prec, flush=True)
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    monkeypatch.setenv("DMRG_HEFF_KCHUNK", "300")
    prob = case(name)
    ref_h = device_plan(ctx, prob, prec)
    if mode == "resident":
        h = streamed_plan(ctx, prob, 2 * pool_bytes(prob) + (1 << 20), prec)
    else:
        slot_kb = pool_bytes(prob) // 1024 + 1  # larger than any wave's blocks
        monkeypatch.setenv("DMRG_HEFF_STREAM_RESIDENT_KB", "0")
        monkeypatch.setenv("DMRG_HEFF_STREAM_SLOT_KB", str(slot_kb))
        h = streamed_plan(ctx, prob, 2 * slot_kb * 1024, prec)
    res_b, str_b, res_w, str_w = h.stream_info()
    print("stream info", res_b, str_b, res_w, str_w, flush=True)
    if mode == "resident":
        assert str_b == 0 and str_w == 0 and res_w >= 1
    else:
        assert res_b == 0 and res_w == 0 and str_w >= 1 and str_b > 0
    for x in inputs(prob):
        y_ref = ref_h.apply(x)
        y = h.apply(x)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
    assert torch.equal(h.diag(), ref_h.diag())


@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_streaming_parity(ctx, name, monkeypatch):
    print("case stream mixed", name, flush=True)
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    prob = case(name)
    third_kb = pool_bytes(prob) // 3 // 1024
    monkeypatch.setenv("DMRG_HEFF_STREAM_RESIDENT_KB", str(third_kb))
    monkeypatch.setenv("DMRG_HEFF_STREAM_SLOT_KB", "1")  # raised to the largest pair's blocks
    h = streamed_plan(ctx, prob, 4 * pool_bytes(prob) + (1 << 20))
    res_b, str_b, res_w, str_w = h.stream_info()
    print("stream info", res_b, str_b, res_w, str_w, flush=True)
    assert str_w >= 3 and str_b > 0
    assert res_b <= third_kb * 1024
    ref_h = device_plan(ctx, prob)
    for i, x in enumerate(inputs(prob)):
        y = h.apply(x)
        y_ref = ref_h.apply(x)
        torch.cuda.synchronize()
        assert rel(y.cpu().numpy(), y_ref.cpu().numpy()) <= 1e-12
        if i == 0:
            assert rel(y.cpu().numpy(), heff_apply(prob)) <= 1e-12
    assert torch.equal(h.diag(), ref_h.diag())


def test_streamed_davidson(monkeypatch):
    """On a non-null stream (the reference solve replays stage graphs; the
    streamed one runs its stages eagerly, as the library decides)."""
    from paper_2407_07411_amd.heff import Context, davidson
    print("case stream davidson", flush=True)
    monkeypatch.setenv("DMRG_HEFF_WORKSPACE_MB", "4")
    prob = _l24(1)
    monkeypatch.setenv("DMRG_HEFF_STREAM_RESIDENT_KB", str(pool_bytes(prob) // 2 // 1024))
    monkeypatch.setenv("DMRG_HEFF_STREAM_SLOT_KB", "2048")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    out = []
    with torch.cuda.stream(stream):
        ctx = Context(0)
        h = streamed_plan(ctx, prob, 4 * pool_bytes(prob))
        assert h.stream_info()[3] >= 2
        ref_h = device_plan(ctx, prob)
        for plan in (ref_h, h):
            psi = prob.psi.to("cuda").clone()
            r = davidson(plan, psi, tol=1e-8, max_iter=80, start_from_diag=True, use_graph=True)
            out.append(r)
    torch.cuda.synchronize()
    print([(r["energy"], r["iters"], r["residual"]) for r in out], flush=True)
    assert out[0]["converged"] and out[1]["converged"]
    assert abs(out[0]["energy"] - out[1]["energy"]) < 1e-10


def _raw_create(ctx, prob, lp, rp, device_bytes):
    """dmrg_heff_create_streamed through ctypes with the given pool pointers."""
    from paper_2407_07411_amd._lib import Term, lib
    from paper_2407_07411_amd.heff import Basis
    L, R = Basis(ctx, prob.Lq, prob.Ld), Basis(ctx, prob.Rq, prob.Rd)
    arr = (Term * len(prob.terms))()
    keep = []
    for i, t in enumerate(prob.terms):
        x = arr[i]
        x.dq[0], x.dq[1] = int(t.dq[0]), int(t.dq[1])
        x.odd, x.hc, x.one_sided, x.reserved = int(t.odd), int(t.hc), int(t.one_sided), 0
        x.coeff = float(t.coeff)
        for side, fld in ((t.left_off, "left_off"), (t.right_off, "right_off")):
            if side is None:
                setattr(x, fld, ctypes.POINTER(ctypes.c_int64)())
            else:
                a = np.ascontiguousarray(np.asarray(side, dtype=np.int64))
                keep.append(a)
                setattr(x, fld, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    q = (ctypes.c_int32 * 2)(int(prob.Q[0]), int(prob.Q[1]))
    h = ctypes.c_void_p()
    st = lib().dmrg_heff_create_streamed(ctx.h, L.h, R.h, q, len(prob.terms), arr, lp[0], lp[1], rp[0], rp[1],
                                          0, int(device_bytes), ctypes.byref(h))
    if st == 0:
        lib().dmrg_heff_destroy(h)
    return st, lib().dmrg_last_error().decode()


def test_refusals(ctx, monkeypatch):
    from paper_2407_07411_amd._lib import DmrgError
    print("case stream refusals", flush=True)
    prob = case("tiny")
    nl, nr = prob.left_pool.numel(), prob.right_pool.numel()
    big = 4 * pool_bytes(prob) + (1 << 20)
    pageable_l = prob.left_pool.contiguous().clone()
    pageable_r = prob.right_pool.contiguous().clone()
    st, msg = _raw_create(ctx, prob, (pageable_l.data_ptr(), nl), (pageable_r.data_ptr(), nr), big)
    assert st == -1 and "pinned" in msg
    dl, dr = prob.left_pool.to("cuda"), prob.right_pool.to("cuda")
    st, msg = _raw_create(ctx, prob, (dl.data_ptr(), nl), (dr.data_ptr(), nr), big)
    assert st == -1 and "pinned" in msg
    pl, pr = pinned(prob.left_pool), pinned(prob.right_pool)
    monkeypatch.setenv("DMRG_HEFF_STREAM_RESIDENT_KB", "0")
    st, msg = _raw_create(ctx, prob, (pl.data_ptr(), nl), (pr.data_ptr(), nr), 64)
    assert st == -3 and "staging" in msg
    st, _ = _raw_create(ctx, prob, (pl.data_ptr(), nl), (pr.data_ptr(), nr), big)
    assert st == 0
    h = streamed_plan(ctx, prob, big)
    x = prob.psi.to("cuda")
    y = torch.empty_like(x)
    for call in (lambda: h.use_graph(True), lambda: h.set_persistent(True), lambda: h.autotune(x, y),
                 lambda: h.apply_profiled(x, y),
                 lambda: h.adjoint(x, x, psibar=torch.zeros_like(x))):
        with pytest.raises(DmrgError) as e:
            call()
        assert e.value.status == -6
    # the plan still works after the refused calls
    assert rel(h.apply(x).cpu().numpy(), heff_apply(prob)) <= 1e-12

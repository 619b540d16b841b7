"""Python binding of the HIP effective-Hamiltonian library.

Argument marshalling only: tensors are handed to the C ABI as raw device
pointers, torch's current HIP stream is the stream every call runs on, and
every number is computed by the library's kernels.  Nothing here falls back
to a CPU implementation: without the built library the calls raise.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

import numpy as np
import torch

from ._lib import (FP32, FP64, SPLIT_BF16X3, DavOpts, DavResult, DmrgError, Term, TermSU2, check, lib)

__all__ = ["Context", "Heff", "HeffSU2", "HeffApply", "davidson", "svd_truncate", "su2_weight",
           "wfn_layout_su2", "FP64", "SPLIT_BF16X3", "FP32", "DmrgError"]


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on a HIP device")
    return t


class Context:
    """A library context on one device, bound to torch's current stream."""

    def __init__(self, device=None):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        h = c_void_p()
        check(lib().dmrg_ctx_create(dev.index, c_void_p(torch.cuda.current_stream(dev).cuda_stream), byref(h)))
        self.h = h
        self._destroy = lib().dmrg_ctx_destroy

    def sync_stream(self):
        check(lib().dmrg_ctx_set_stream(self.h, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    def __del__(self):
        # the destroy entry point is bound at construction: module globals
        # may already be gone when the interpreter shuts down
        fn = getattr(self, "_destroy", None)
        if getattr(self, "h", None) and fn is not None:
            fn(self.h)
            self.h = None


class Basis:
    def __init__(self, ctx: Context, qn, dim):
        qn = np.ascontiguousarray(np.asarray(qn, dtype=np.int32).reshape(-1, 2))
        dim = np.ascontiguousarray(np.asarray(dim, dtype=np.int64).reshape(-1))
        self.qn, self.dim, self.ctx = qn, dim, ctx
        h = c_void_p()
        check(lib().dmrg_basis_create(ctx.h, int(len(dim)), qn.ctypes.data_as(ctypes.POINTER(c_int32)),
                                      dim.ctypes.data_as(ctypes.POINTER(c_int64)), byref(h)))
        self.h = h
        self._destroy = lib().dmrg_basis_destroy

    def __del__(self):
        # the destroy entry point is bound at construction: module globals
        # may already be gone when the interpreter shuts down
        fn = getattr(self, "_destroy", None)
        if getattr(self, "h", None) and fn is not None:
            fn(self.h)
            self.h = None


def wfn_layout(L: Basis, R: Basis, Q):
    q = (c_int32 * 2)(int(Q[0]), int(Q[1]))
    nb, total = c_int64(), c_int64()
    offs = np.zeros(len(L.dim), dtype=np.int64)
    check(lib().dmrg_wfn_layout(L.h, R.h, q, byref(nb), offs.ctypes.data_as(ctypes.POINTER(c_int64)), byref(total)))
    return int(nb.value), offs, int(total.value)


def _pinned_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.device.type == "cpu" and t.is_pinned()
            and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor in pinned host memory")
    return t


class Heff:
    """H_eff of one two-site step: sector tables, operator-pair terms and the
    two operator pools (borrowed: they must stay alive and unchanged).

    device_bytes=None: the pools are device tensors.  Otherwise they are
    pinned host tensors (out-of-core form) and device_bytes bounds the device
    memory for their blocks: what fits is copied once, the rest is streamed
    through two staging slots on every apply."""

    def __init__(self, ctx: Context, Lq, Ld, Rq, Rd, Q, terms, left_pool, right_pool, prec=FP64,
                 device_bytes=None):
        self.ctx = ctx
        self.L = Basis(ctx, Lq, Ld)
        self.R = Basis(ctx, Rq, Rd)
        conv = _dev_f64 if device_bytes is None else _pinned_f64
        self.left_pool = conv(left_pool, "left_pool")
        self.right_pool = conv(right_pool, "right_pool")
        nL, nR = len(self.L.dim), len(self.R.dim)
        arr = (Term * max(1, len(terms)))()
        keep = []
        for i, t in enumerate(terms):
            x = arr[i]
            x.dq[0], x.dq[1] = int(t.dq[0]), int(t.dq[1])
            x.odd, x.hc, x.one_sided, x.reserved = int(t.odd), int(t.hc), int(t.one_sided), 0
            x.coeff = float(t.coeff)
            for side, n, fld in ((t.left_off, nL, "left_off"), (t.right_off, nR, "right_off")):
                if side is None:
                    setattr(x, fld, ctypes.POINTER(c_int64)())
                else:
                    a = np.ascontiguousarray(np.asarray(side, dtype=np.int64).reshape(-1))
                    if a.size != n:
                        raise ValueError(f"term {i}: {fld} has {a.size} entries, expected {n}")
                    keep.append(a)
                    setattr(x, fld, a.ctypes.data_as(ctypes.POINTER(c_int64)))
        q = (c_int32 * 2)(int(Q[0]), int(Q[1]))
        self.Q = (int(Q[0]), int(Q[1]))
        ctx.sync_stream()
        h = c_void_p()
        if device_bytes is None:
            check(lib().dmrg_heff_create(ctx.h, self.L.h, self.R.h, q, len(terms), arr,
                                         _ptr(self.left_pool), self.left_pool.numel(),
                                         _ptr(self.right_pool), self.right_pool.numel(), int(prec), byref(h)))
        else:
            check(lib().dmrg_heff_create_streamed(ctx.h, self.L.h, self.R.h, q, len(terms), arr,
                                                  _ptr(self.left_pool), self.left_pool.numel(),
                                                  _ptr(self.right_pool), self.right_pool.numel(), int(prec),
                                                  int(device_bytes), byref(h)))
        self.h = h
        self._destroy = lib().dmrg_heff_destroy
        self.size = int(lib().dmrg_heff_size(h))

    def __del__(self):
        # the destroy entry point is bound at construction: module globals
        # may already be gone when the interpreter shuts down
        fn = getattr(self, "_destroy", None)
        if getattr(self, "h", None) and fn is not None:
            fn(self.h)
            self.h = None

    def stream_info(self):
        """(resident bytes, bytes streamed per apply, resident waves, streamed
        waves) of the out-of-core form; zeros for device pools."""
        rb, sb, rw, sw = c_int64(), c_int64(), c_int32(), c_int32()
        check(lib().dmrg_heff_stream_info(self.h, byref(rb), byref(sb), byref(rw), byref(sw)))
        return int(rb.value), int(sb.value), int(rw.value), int(sw.value)

    def set_precision(self, prec):
        check(lib().dmrg_heff_set_precision(self.h, int(prec)))

    def set_persistent(self, enable=True):
        """FP64 matvec as one persistent launch (bit-identical results)."""
        check(lib().dmrg_heff_set_persistent(self.h, 1 if enable else 0))

    def check(self):
        """Synchronises; raises if a persistent launch gave up a wait."""
        self.ctx.sync_stream()
        check(lib().dmrg_heff_check(self.h))

    def use_graph(self, enable=True):
        check(lib().dmrg_heff_use_graph(self.h, 1 if enable else 0))

    def flops(self):
        f, b = c_double(), c_double()
        check(lib().dmrg_heff_flops(self.h, byref(f), byref(b)))
        return f.value, b.value

    def workspace_bytes(self):
        return int(lib().dmrg_heff_workspace_bytes(self.h))

    def _vec(self, t, name):
        _dev_f64(t, name)
        if t.numel() != self.size:
            raise ValueError(f"{name} has {t.numel()} elements, expected {self.size}")
        return t

    def apply(self, psi, out=None):
        self._vec(psi, "psi")
        y = torch.empty_like(psi) if out is None else self._vec(out, "out")
        self.ctx.sync_stream()
        check(lib().dmrg_heff_apply(self.h, _ptr(psi), _ptr(y)))
        return y

    def autotune(self, psi, scratch=None, reps=3):
        """Pick the fastest tile shape per problem class on this plan's own
        problems (timed on the device) and rebuild the plan with it."""
        self._vec(psi, "psi")
        y = torch.empty_like(psi) if scratch is None else self._vec(scratch, "scratch")
        self.ctx.sync_stream()
        check(lib().dmrg_heff_autotune(self.h, _ptr(psi), _ptr(y), int(reps)))

    def launches(self):
        """(kernel ids, algorithmic FLOPs) of the matvec's launches."""
        n = c_int64()
        check(lib().dmrg_heff_launches(self.h, byref(n), None, None))
        k = np.zeros(n.value, dtype=np.int32)
        f = np.zeros(n.value, dtype=np.float64)
        check(lib().dmrg_heff_launches(self.h, byref(n), k.ctypes.data_as(ctypes.POINTER(c_int32)),
                                       f.ctypes.data_as(ctypes.POINTER(c_double))))
        return k, f

    def apply_profiled(self, psi, out):
        """Eager matvec with a HIP-event duration (ms) per launch."""
        self._vec(psi, "psi")
        self._vec(out, "out")
        k, _ = self.launches()
        ms = np.zeros(len(k), dtype=np.float32)
        self.ctx.sync_stream()
        check(lib().dmrg_heff_apply_profiled(self.h, _ptr(psi), _ptr(out),
                                             ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return ms

    def diag(self, out=None):
        d = torch.empty(self.size, dtype=torch.float64, device=self.ctx.device) if out is None else self._vec(out, "out")
        self.ctx.sync_stream()
        check(lib().dmrg_heff_diag(self.h, _ptr(d)))
        return d

    def adjoint(self, psi, ybar, psibar=None, left_bar=None, right_bar=None):
        """Accumulates into the given buffers (+=); returns them."""
        self._vec(psi, "psi")
        self._vec(ybar, "ybar")
        if psibar is not None:
            self._vec(psibar, "psibar")
        for t, pool, name in ((left_bar, self.left_pool, "left_bar"), (right_bar, self.right_pool, "right_bar")):
            if t is not None:
                _dev_f64(t, name)
                if t.numel() != pool.numel():
                    raise ValueError(f"{name} must match its pool's length")
        self.ctx.sync_stream()
        check(lib().dmrg_heff_apply_adjoint(self.h, _ptr(psi), _ptr(ybar), _ptr(psibar), _ptr(left_bar),
                                            _ptr(right_bar)))
        return psibar, left_bar, right_bar


def su2_weight(two_ja, two_jc, two_ja2, two_jc2, two_k, two_s):
    """The library's recoupling weight of the SU(2) form (host call)."""
    return float(lib().dmrg_su2_weight(int(two_ja), int(two_jc), int(two_ja2), int(two_jc2), int(two_k),
                                       int(two_s)))


def wfn_layout_su2(L: Basis, R: Basis, Q):
    """(left sector, right sector, offset) of every reduced block and the
    total length of the SU(2) wavefunction."""
    q = (c_int32 * 2)(int(Q[0]), int(Q[1]))
    nb, total = c_int64(), c_int64()
    check(lib().dmrg_wfn_layout_su2(L.h, R.h, q, byref(nb), None, None, None, byref(total)))
    bl = np.zeros(nb.value, dtype=np.int32)
    br = np.zeros(nb.value, dtype=np.int32)
    bo = np.zeros(nb.value, dtype=np.int64)
    check(lib().dmrg_wfn_layout_su2(L.h, R.h, q, byref(nb), bl.ctypes.data_as(c_void_p),
                                    br.ctypes.data_as(c_void_p), bo.ctypes.data_as(c_void_p), byref(total)))
    return bl, br, bo, int(total.value)


class HeffSU2(Heff):
    """H_eff in the SU(2) spin-adapted form: sectors (N, 2j) with multiplet
    counts, total Q = (N, 2S), terms with a spin rank and reduced blocks
    listed as (output sector, input sector, offset) rows; the same device
    pools and calls as Heff."""

    def __init__(self, ctx: Context, Lq, Ld, Rq, Rd, Q, terms, left_pool, right_pool, prec=FP64):
        self.ctx = ctx
        self.L = Basis(ctx, Lq, Ld)
        self.R = Basis(ctx, Rq, Rd)
        self.left_pool = _dev_f64(left_pool, "left_pool")
        self.right_pool = _dev_f64(right_pool, "right_pool")
        arr = (TermSU2 * max(1, len(terms)))()
        keep = []
        for i, t in enumerate(terms):
            x = arr[i]
            x.two_k, x.dn, x.odd, x.hc = int(t.two_k), int(t.dn), int(t.odd), int(t.hc)
            x.one_sided, x.reserved, x.coeff = int(t.one_sided), 0, float(t.coeff)
            for tab, nfld, pfld in ((t.left_blocks, "n_left", "left_blocks"),
                                    (t.right_blocks, "n_right", "right_blocks")):
                if tab is None:
                    setattr(x, nfld, 0)
                    setattr(x, pfld, ctypes.POINTER(c_int64)())
                else:
                    a = np.ascontiguousarray(np.asarray(tab, dtype=np.int64).reshape(-1, 3))
                    keep.append(a)
                    setattr(x, nfld, a.shape[0])
                    setattr(x, pfld, a.ctypes.data_as(ctypes.POINTER(c_int64)))
        q = (c_int32 * 2)(int(Q[0]), int(Q[1]))
        self.Q = (int(Q[0]), int(Q[1]))
        ctx.sync_stream()
        h = c_void_p()
        check(lib().dmrg_heff_create_su2(ctx.h, self.L.h, self.R.h, q, len(terms), arr,
                                         _ptr(self.left_pool), self.left_pool.numel(),
                                         _ptr(self.right_pool), self.right_pool.numel(), int(prec), byref(h)))
        self.h = h
        self._destroy = lib().dmrg_heff_destroy
        self.size = int(lib().dmrg_heff_size(h))


class HeffApply(torch.autograd.Function):
    """y = H_eff(left_pool, right_pool) psi with the hand-written adjoint.

    The backward recomputes the two-GEMM intermediates instead of keeping
    them from the forward pass."""

    @staticmethod
    def forward(ctx, psi, left_pool, right_pool, heff: Heff):
        if left_pool.data_ptr() != heff.left_pool.data_ptr() or right_pool.data_ptr() != heff.right_pool.data_ptr():
            raise ValueError("pools must be the tensors the Heff plan was built on")
        ctx.heff = heff
        psi_c = psi.contiguous()
        ctx.save_for_backward(psi_c)
        return heff.apply(psi_c)

    @staticmethod
    def backward(ctx, ybar):
        (psi,) = ctx.saved_tensors
        h = ctx.heff
        ybar = ybar.contiguous()
        need_psi, need_l, need_r = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gp = torch.zeros_like(psi) if need_psi else None
        gl = torch.zeros_like(h.left_pool) if need_l else None
        gr = torch.zeros_like(h.right_pool) if need_r else None
        if need_psi or need_l or need_r:
            h.adjoint(psi, ybar, gp, gl, gr)
        return gp, gl, gr, None


def davidson(heff: Heff, psi, tol=1e-8, max_iter=200, max_subspace=24, restart_keep=2, use_graph=False,
             fp64_tail=0, start_from_diag=False):
    """Lowest eigenpair of H_eff on the device; psi (start vector, ignored
    with start_from_diag) is overwritten by the Ritz vector.  Returns a dict
    of the solver result."""
    heff._vec(psi, "psi")
    opts = DavOpts(int(max_iter), int(max_subspace), int(restart_keep), 1 if use_graph else 0, float(tol),
                   int(fp64_tail), 1 if start_from_diag else 0)
    res = DavResult()
    heff.ctx.sync_stream()
    st = lib().dmrg_davidson(heff.h, _ptr(psi), byref(opts), byref(res))
    if st not in (0, -5):
        check(st)
    return dict(energy=res.energy, residual=res.residual, iters=res.iters, matvecs=res.matvecs,
                converged=bool(res.converged), tail_iters=res.tail_iters, split_iters=res.split_iters,
                split_residual=res.split_residual, split_energy=res.split_energy, status=st)


def svd_truncate(ctx: Context, Lq, Ld, Rq, Rd, Q, psi, max_keep, cutoff=0.0, out=None, noalloc=False):
    """Block-wise SVD of psi with global truncation.  Returns (kept_dim,
    U, S, Vt, trunc_err) with the factors packed per left sector.  out: an
    optional (U, S, Vt) of device buffers to write into.  noalloc: run the
    library's allocation-free variant (temporaries in its per-device scratch
    array)."""
    L, R = Basis(ctx, Lq, Ld), Basis(ctx, Rq, Rd)
    _dev_f64(psi, "psi")
    Ld, Rd = L.dim, R.dim
    _, offs, total = wfn_layout(L, R, Q)
    if psi.numel() != total:
        raise ValueError("psi does not match the layout")
    ucap = scap = vcap = 0
    for a in range(len(Ld)):
        if offs[a] < 0:
            continue
        qa = L.qn[a]
        c = [i for i in range(len(Rd)) if R.qn[i][0] == Q[0] - qa[0] and R.qn[i][1] == Q[1] - qa[1]][0]
        k = min(Ld[a], Rd[c])
        ucap += Ld[a] * k
        scap += k
        vcap += k * Rd[c]
    dev = ctx.device
    if out is None:
        U = torch.empty(max(1, ucap), dtype=torch.float64, device=dev)
        S = torch.empty(max(1, scap), dtype=torch.float64, device=dev)
        Vt = torch.empty(max(1, vcap), dtype=torch.float64, device=dev)
    else:
        U, S, Vt = (_dev_f64(t, n) for t, n in zip(out, ("U", "S", "Vt")))
    kept = np.zeros(len(Ld), dtype=np.int64)
    err = c_double()
    q = (c_int32 * 2)(int(Q[0]), int(Q[1]))
    ctx.sync_stream()
    fn = lib().dmrg_svd_truncate_noalloc if noalloc else lib().dmrg_svd_truncate
    check(fn(ctx.h, L.h, R.h, q, _ptr(psi), int(max_keep), float(cutoff),
                                  kept.ctypes.data_as(ctypes.POINTER(c_int64)), _ptr(U), U.numel(), _ptr(S),
                                  S.numel(), _ptr(Vt), Vt.numel(), byref(err)))
    return kept, U, S, Vt, err.value

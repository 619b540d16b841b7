"""Binding of the operator-block chain: the ab initio Hamiltonian on an
orbital chain and the two-site DMRG sweep (argument marshalling only)."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p
from types import SimpleNamespace

import numpy as np

from ._lib import DavOpts, DavResult, check, lib


def _p(a):
    return a.ctypes.data_as(c_void_p)


class Chain:
    """Operator blocks for integrals h (L x L) and V (L^4, chemists'), n_elec
    electrons with 2Sz = two_sz, at most D states per block."""

    def __init__(self, ctx, h, V, n_elec, two_sz, D, seed=0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        L = h.shape[0]
        assert h.shape == (L, L) and V.shape == (L,) * 4
        self.L, self.ctx = L, ctx
        self.Q = (int(n_elec), int(two_sz))
        out = c_void_p()
        check(lib().dmrg_chain_create(ctx.h if ctx is not None else None, L, _p(h), _p(V), int(n_elec),
                                      int(two_sz), int(D), int(seed), byref(out)))
        self.h = out
        self._destroy = lib().dmrg_chain_destroy

    def __del__(self):
        # the destroy entry point is bound at construction: module globals
        # may already be gone when the interpreter shuts down
        fn = getattr(self, "_destroy", None)
        if getattr(self, "h", None) and fn is not None:
            fn(self.h)
            self.h = None

    def step(self, l, direction, tol=1e-8, max_iter=200, max_subspace=24, restart_keep=2):
        opts = DavOpts(int(max_iter), int(max_subspace), int(restart_keep), 0, float(tol), 0, 0)
        e, err, res = c_double(), c_double(), DavResult()
        if self.ctx is not None:
            self.ctx.sync_stream()
        check(lib().dmrg_chain_step(self.h, int(l), int(direction), byref(opts), byref(e), byref(err),
                                    byref(res)))
        return dict(energy=e.value, trunc_err=err.value, iters=res.iters, residual=res.residual,
                    converged=bool(res.converged))

    def sweep(self, direction, **kw):
        """One sweep (+1: left to right, -1: right to left); per-step results."""
        sites = range(self.L - 1) if direction > 0 else range(self.L - 2, -1, -1)
        return [dict(site=l, **self.step(l, direction, **kw)) for l in sites]

    def grow_left(self, l):
        """Build the left blocks up to [0, l) without truncation (host only)."""
        check(lib().dmrg_chain_grow_left(self.h, int(l)))

    def export(self, l):
        """The two-site problem at (l, l+1) as host arrays (no device needed)."""
        L_ = lib()
        nl, nr = c_int32(), c_int32()
        nt, lp, rp = c_int64(), c_int64(), c_int64()
        check(L_.dmrg_chain_export(self.h, int(l), byref(nl), byref(nr), byref(nt), byref(lp), byref(rp),
                                   None, None, None, None, None, None, None, None, None))
        lqn = np.zeros((nl.value, 2), dtype=np.int32)
        ldim = np.zeros(nl.value, dtype=np.int64)
        rqn = np.zeros((nr.value, 2), dtype=np.int32)
        rdim = np.zeros(nr.value, dtype=np.int64)
        info = np.zeros((nt.value, 4), dtype=np.int32)
        loff = np.zeros((nt.value, nl.value), dtype=np.int64)
        roff = np.zeros((nt.value, nr.value), dtype=np.int64)
        lpool = np.zeros(max(lp.value, 1))
        rpool = np.zeros(max(rp.value, 1))
        check(L_.dmrg_chain_export(self.h, int(l), byref(nl), byref(nr), byref(nt), byref(lp), byref(rp),
                                   _p(lqn), _p(ldim), _p(rqn), _p(rdim), _p(info), _p(loff), _p(roff),
                                   _p(lpool), _p(rpool)))
        terms = []
        for t in range(nt.value):
            one = int(info[t, 3])
            terms.append(SimpleNamespace(dq=(int(info[t, 0]), int(info[t, 1])), odd=int(info[t, 2]), hc=0,
                                         one_sided=one, coeff=1.0,
                                         left_off=None if one == 2 else loff[t].copy(),
                                         right_off=None if one == 1 else roff[t].copy()))
        return SimpleNamespace(Lq=lqn, Ld=ldim, Rq=rqn, Rd=rdim, Q=np.array(self.Q, dtype=np.int32),
                               terms=terms, left_pool=lpool, right_pool=rpool)

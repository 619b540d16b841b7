"""Adjoint of the operator-sum matvec (oracle; test infrastructure).

For y = H_eff(O) psi and an upstream gradient ybar, the loss f = <ybar, y>
is bilinear.  Per contribution Y_b += alpha * op(A) X op(B)^T (X the input
block, op = identity or transpose of the stored block):

  psibar_in      += alpha * op(A)^T ybar_out op(B)
  d f / d op(A)   = alpha * ybar_out op(B) X^T
  d f / d op(B)   = alpha * ybar_out^T op(A) X

and the stored block's gradient is that matrix, transposed when the stored
block entered transposed (hermitian-conjugate partner terms).  One-sided
terms drop the missing factor.  These are the contractions an orbital
gradient (DMRG-CASSCF, mentioned in the P450 section of the paper) needs.
"""
from __future__ import annotations

import numpy as np

from .heff import _get, _np, layout_of, term_items


def heff_adjoint(prob, psi, ybar):
    lay = layout_of(prob)
    lp = _np(prob.left_pool).astype(np.float64)
    rp = _np(prob.right_pool).astype(np.float64)
    pools = {"L": lp, "R": rp}
    x = _np(psi).astype(np.float64)
    yb = _np(ybar).astype(np.float64)
    psibar = np.zeros(lay.total)
    gL = np.zeros_like(lp)
    gR = np.zeros_like(rp)
    grads = {"L": gL, "R": gR}
    for t in prob.terms:
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            X = lay.block(x, a)
            Yb = lay.block(yb, b)
            opA = None if A is None else _get(pools, A, tA)
            opB = None if B is None else _get(pools, B, tB)
            # psi gradient
            G = Yb if opA is None else opA.T @ Yb
            if opB is not None:
                G = G @ opB
            lay.block(psibar, a)[...] += alpha * G
            # left operator gradient
            if opA is not None:
                M = Yb if opB is None else Yb @ opB
                gA = alpha * (M @ X.T)
                kind, off, rows, cols = A
                tgt = grads[kind][off:off + rows * cols].reshape(rows, cols)
                tgt += gA.T if tA else gA
            if opB is not None:
                M = Yb.T if opA is None else Yb.T @ opA
                gB = alpha * (M @ X)
                kind, off, rows, cols = B
                tgt = grads[kind][off:off + rows * cols].reshape(rows, cols)
                tgt += gB.T if tB else gB
    return psibar, gL, gR

"""Operator-sum two-site effective Hamiltonian, plain definition (oracle).

Test infrastructure only.  The paper solves the local eigenproblem of each
DMRG update with Lanczos or Davidson (Numerical procedure section); the
operator applied there is the two-site effective Hamiltonian, written in
the normal/complementary operator form of ab initio DMRG as a sum of
left-block x right-block operator pairs:

    H_eff = sum_xi c_xi (O^L_xi (x) O^R_xi) with a fermionic sign.

The two-site wavefunction is block sparse: block Psi[q, Q-q] couples
enlarged-left sector q with enlarged-right sector Q-q and is stored
row-major.  For one term and one input block,

    Y[q+dq, Q-q-dq] += c * s * O^L[q+dq, q] @ Psi[q, Q-q] @ O^R[Q-q-dq, Q-q]^T

where s = (-1)^{N(q)} when the right operator changes the particle number by
an odd amount (moving it past the left state, Jordan-Wigner order left
before right) and s = 1 otherwise.  A term flagged `hc` also contributes its
hermitian conjugate (O^L^T (x) O^R^T) with coefficient (-1)^odd * c, the
sign again read from that partner's input left sector.

This module multiplies every pair left-first, in ascending term order, with
numpy matmuls in float64; it knows nothing about tiling, batching or
association order.
"""
from __future__ import annotations

import numpy as np


def _np(x):
    if hasattr(x, "detach"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


class Layout:
    """Block structure of the two-site wavefunction (its own decoding)."""

    def __init__(self, Lq, Ld, Rq, Rd, Q):
        self.Lq = np.asarray(Lq).reshape(-1, 2)
        self.Rq = np.asarray(Rq).reshape(-1, 2)
        self.Ld = np.asarray(Ld, dtype=np.int64)
        self.Rd = np.asarray(Rd, dtype=np.int64)
        self.Q = np.asarray(Q).reshape(2)
        self.lidx = {tuple(q): i for i, q in enumerate(self.Lq.tolist())}
        self.ridx = {tuple(q): i for i, q in enumerate(self.Rq.tolist())}
        self.partner = {}   # left sector a -> right sector c
        self.offset = {}    # left sector a -> offset of block (a, c)
        off = 0
        for a, q in enumerate(self.Lq.tolist()):
            c = self.ridx.get((int(self.Q[0]) - q[0], int(self.Q[1]) - q[1]))
            if c is None:
                continue
            self.partner[a] = c
            self.offset[a] = off
            off += int(self.Ld[a] * self.Rd[c])
        self.total = off

    def block(self, vec, a):
        c = self.partner[a]
        o = self.offset[a]
        return vec[o:o + int(self.Ld[a] * self.Rd[c])].reshape(int(self.Ld[a]), int(self.Rd[c]))

    def shift_left(self, a, dq, sign=+1):
        q = self.Lq[a]
        return self.lidx.get((int(q[0]) + sign * dq[0], int(q[1]) + sign * dq[1]))

    def shift_right(self, c, dq, sign=+1):
        r = self.Rq[c]
        return self.ridx.get((int(r[0]) - sign * dq[0], int(r[1]) - sign * dq[1]))


def layout_of(prob):
    return Layout(prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q)


def _left_block(pool, off, rows, cols):
    return pool[off:off + rows * cols].reshape(rows, cols)


def term_items(lay: Layout, t):
    """All (input a, output b, A, transA, B, transB, alpha) of one term.

    A and B are (pool-kind, offset, rows, cols) of the STORED blocks;
    trans flags say whether the stored block is applied transposed.
    Missing blocks (offset -1) or blocks whose wavefunction partner does not
    exist produce no item.
    """
    items = []
    for a in lay.partner:
        c = lay.partner[a]
        q_n = int(lay.Lq[a][0])
        s = -1.0 if (t.odd and q_n % 2) else 1.0
        # One-sided terms are particle-number conserving (even), so their
        # hermitian-conjugate partner is the transposed block with +c.
        if t.one_sided == 1:
            off = int(t.left_off[a])
            if off >= 0:
                A = ("L", off, int(lay.Ld[a]), int(lay.Ld[a]))
                items.append((a, a, A, False, None, False, t.coeff))
                if t.hc:
                    items.append((a, a, A, True, None, False, t.coeff))
            continue
        if t.one_sided == 2:
            off = int(t.right_off[c])
            if off >= 0:
                B = ("R", off, int(lay.Rd[c]), int(lay.Rd[c]))
                items.append((a, a, None, False, B, False, t.coeff))
                if t.hc:
                    items.append((a, a, None, False, B, True, t.coeff))
            continue
        b = lay.shift_left(a, t.dq)
        if b is None or b not in lay.partner:
            continue
        e = lay.partner[b]
        if lay.shift_right(c, t.dq) != e:
            continue
        lo, ro = int(t.left_off[a]), int(t.right_off[c])
        if lo < 0 or ro < 0:
            continue
        A = ("L", lo, int(lay.Ld[b]), int(lay.Ld[a]))
        B = ("R", ro, int(lay.Rd[e]), int(lay.Rd[c]))
        items.append((a, b, A, False, B, False, t.coeff * s))
        if t.hc:
            s2 = -1.0 if (t.odd and int(lay.Lq[b][0]) % 2) else 1.0
            c2 = -t.coeff if t.odd else t.coeff
            items.append((b, a, A, True, B, True, c2 * s2))
    return items


def _get(pools, spec, trans):
    kind, off, rows, cols = spec
    m = pools[kind][off:off + rows * cols].reshape(rows, cols)
    return m.T if trans else m


def heff_apply(prob, psi=None, terms=None, left_pool=None, right_pool=None, out_left_sectors=None):
    """y = H_eff psi, plain definition, float64, left-first, ascending terms.

    out_left_sectors (optional set of left-sector indices) restricts the
    computation to those output blocks; the other blocks stay zero."""
    lay = layout_of(prob)
    pools = {"L": _np(prob.left_pool if left_pool is None else left_pool),
             "R": _np(prob.right_pool if right_pool is None else right_pool)}
    x = _np(prob.psi if psi is None else psi).astype(np.float64)
    y = np.zeros(lay.total)
    for t in (prob.terms if terms is None else terms):
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            if out_left_sectors is not None and b not in out_left_sectors:
                continue
            X = lay.block(x, a)
            Yb = lay.block(y, b)
            if A is not None:
                X = _get(pools, A, tA) @ X
            if B is not None:
                X = X @ _get(pools, B, tB).T
            Yb += alpha * X
    return y


def heff_dense(prob, terms=None):
    """Dense H_eff by brute force: apply the matvec to every unit vector."""
    lay = layout_of(prob)
    n = lay.total
    H = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        H[:, j] = heff_apply(prob, e, terms=terms)
    return H


def heff_diag(prob):
    """diag(H_eff): only dq = 0 terms reach the diagonal; for those
    diag(A Psi B^T) at (i, j) is A_ii * B_jj (transposes keep the diagonal)."""
    lay = layout_of(prob)
    pools = {"L": _np(prob.left_pool), "R": _np(prob.right_pool)}
    d = np.zeros(lay.total)
    for t in prob.terms:
        if tuple(t.dq) != (0, 0):
            continue
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            assert a == b
            c = lay.partner[a]
            da = np.ones(int(lay.Ld[a])) if A is None else np.diag(_get(pools, A, tA))
            db = np.ones(int(lay.Rd[c])) if B is None else np.diag(_get(pools, B, tB))
            lay.block(d, a)[...] += alpha * np.outer(da, db)
    return d


def count_flops(prob):
    """Algorithmic FLOPs of one matvec: every (term, block) pair, hc partners
    included, at the cheaper association order; one-sided terms one GEMM."""
    lay = layout_of(prob)
    total = 0
    for t in prob.terms:
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            c, e = lay.partner[a], lay.partner[b]
            dl, dl2, dr, dr2 = int(lay.Ld[a]), int(lay.Ld[b]), int(lay.Rd[c]), int(lay.Rd[e])
            if B is None:
                total += 2 * dl2 * dl * dr
            elif A is None:
                total += 2 * dl * dr * dr2
            else:
                total += min(2 * dl2 * dl * dr + 2 * dl2 * dr * dr2,
                             2 * dl * dr * dr2 + 2 * dl2 * dl * dr2)
    return total


def count_bytes(prob):
    """Algorithmic bytes of one matvec: every stored operator block that some
    (term, block) pair uses, read once (a block shared by several terms or by
    a term and its hermitian-conjugate partner counts once), plus psi read
    and y written; 8 bytes per double."""
    lay = layout_of(prob)
    used = {}
    for t in prob.terms:
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            for spec in (A, B):
                if spec is not None:
                    kind, off, rows, cols = spec
                    used[(kind, off)] = rows * cols
    return 8 * (sum(used.values()) + 2 * lay.total)


def _stored_rows(pool, spec, trans, rows):
    """Rows `rows` of a stored block, or of its transpose, as float64 numpy.
    The pool may be a numpy array or a (device) tensor: only the needed
    slices are copied."""
    kind, off, nr, nc = spec
    out = []
    for r in rows:
        if not trans:
            v = pool[off + r * nc: off + (r + 1) * nc]
        else:
            v = pool[off + r: off + nr * nc: nc]
        out.append(_np(v).astype(np.float64))
    return np.stack(out) if out else np.zeros((0, nr if trans else nc))


def heff_entries(prob, b, rows, cols, psi=None):
    """Entries y[b][rows][:, cols] of y = H_eff psi by the same definition as
    heff_apply (left sector b of the output; row and column indices inside
    that block), plus the sum of the absolute values of every product that
    enters each entry (the scale of its rounding error).

    Per item: (A[rows, :] @ Psi_a) @ B[cols, :]^T, so a whole-size problem can
    be sampled without forming any full output block."""
    lay = layout_of(prob)
    pools = {"L": prob.left_pool, "R": prob.right_pool}
    x = _np(prob.psi if psi is None else psi).astype(np.float64)
    rows, cols = list(rows), list(cols)
    val = np.zeros((len(rows), len(cols)))
    mag = np.zeros((len(rows), len(cols)))
    for t in prob.terms:
        for (a, bb, A, tA, B, tB, alpha) in term_items(lay, t):
            if bb != b:
                continue
            X = lay.block(x, a)
            XA = X[rows, :] if A is None else _stored_rows(pools[A[0]], A, tA, rows) @ X
            XAabs = np.abs(X[rows, :]) if A is None else np.abs(_stored_rows(pools[A[0]], A, tA, rows)) @ np.abs(X)
            if B is None:
                v, m = XA[:, cols], XAabs[:, cols]
            else:
                Bc = _stored_rows(pools[B[0]], B, tB, cols)
                v, m = XA @ Bc.T, XAabs @ np.abs(Bc).T
            val += alpha * v
            mag += abs(alpha) * m
    return val, mag


def _rows_of(pool, spec, trans, rows_per_item):
    """Rows of op(stored block) for many items of one stored-block shape
    class: spec[i] = (kind, off, nr, nc) with the same row length, rows
    `rows_per_item` (a list of row indices, the same for every item).
    Returns float64 numpy of shape (n_items, len(rows), row_length).  Only
    the needed entries leave the pool (one gather per call)."""
    offs = np.array([s[1] for s in spec], dtype=np.int64)
    nr = np.array([s[2] for s in spec], dtype=np.int64)
    nc = np.array([s[3] for s in spec], dtype=np.int64)
    tr = np.array(trans, dtype=bool)
    r = np.asarray(rows_per_item, dtype=np.int64)
    length = np.where(tr, nr, nc)
    assert np.all(length == length[0])
    k = np.arange(int(length[0]), dtype=np.int64)
    # not transposed: element (r, k) of the stored block at off + r * nc + k
    # transposed:     element (k, r) of the stored block at off + k * nc + r
    start = offs[:, None] + np.where(tr[:, None], r[None, :], r[None, :] * nc[:, None])
    step = np.where(tr, nc, 1)
    idx = start[:, :, None] + step[:, None, None] * k[None, None, :]
    if hasattr(pool, "detach"):  # a (device) tensor: gather there, copy the entries only
        import torch
        ti = torch.from_numpy(idx.reshape(-1)).to(pool.device)
        return pool.detach().index_select(0, ti).cpu().numpy().astype(np.float64).reshape(idx.shape)
    return np.asarray(pool)[idx].astype(np.float64)


def heff_entries_blocks(prob, samples, psi=None):
    """heff_entries for many output blocks at once: samples maps an output
    left sector b to (rows, cols); returns {b: (val, mag)}.

    Same definition and the same per-item products as heff_entries,
    y_b[rows, cols] = sum over items of alpha * op(A)[rows, :] X_a op(B)[cols, :]^T,
    with the items gathered per (input block, output block, item kind) so
    that each group is one stacked numpy product (the sum over items is
    then taken group by group instead of in term order: an FP64 rounding
    difference only)."""
    lay = layout_of(prob)
    pools = {"L": prob.left_pool, "R": prob.right_pool}
    x = _np(prob.psi if psi is None else psi).astype(np.float64)
    groups = {}
    for t in prob.terms:
        for (a, b, A, tA, B, tB, alpha) in term_items(lay, t):
            if b not in samples:
                continue
            kind = 0 if (A is not None and B is not None) else (1 if B is None else 2)
            groups.setdefault((a, b, kind), []).append((A, tA, B, tB, alpha))
    out = {}
    for b, (rows, cols) in samples.items():
        out[b] = (np.zeros((len(rows), len(cols))), np.zeros((len(rows), len(cols))))
    for (a, b, kind), items in groups.items():
        rows, cols = samples[b]
        rows, cols = list(rows), list(cols)
        X = lay.block(x, a)
        al = np.array([it[4] for it in items])
        if kind != 2:  # op(A)[rows, :] of every item: (n, |rows|, d_L(a))
            A_ = _rows_of(pools["L"], [it[0] for it in items], [it[1] for it in items], rows)
        if kind != 1:  # op(B)[cols, :] of every item: (n, |cols|, d_R(c))
            B_ = _rows_of(pools["R"], [it[2] for it in items], [it[3] for it in items], cols)
        if kind == 0:
            P = (A_.reshape(-1, X.shape[0]) @ X).reshape(len(items), len(rows), -1)
            Pm = (np.abs(A_).reshape(-1, X.shape[0]) @ np.abs(X)).reshape(len(items), len(rows), -1)
            v = np.einsum("nrk,nck->nrc", P, B_)
            m = np.einsum("nrk,nck->nrc", Pm, np.abs(B_))
        elif kind == 1:
            v = A_ @ X[:, cols][None, :, :]
            m = np.abs(A_) @ np.abs(X[:, cols])[None, :, :]
        else:
            v = np.einsum("rk,nck->nrc", X[rows, :], B_)
            m = np.einsum("rk,nck->nrc", np.abs(X[rows, :]), np.abs(B_))
        val, mag = out[b]
        val += np.einsum("n,nrc->rc", al, v)
        mag += np.einsum("n,nrc->rc", np.abs(al), m)
    return out

"""Physical operator pairs of the ab initio Hamiltonian across one cut (oracle).

Test infrastructure only.  The DMRG update of the paper (Numerical
procedure section) acts with the full Hamiltonian H of Eq. 2 on the two-site
space.  Cutting the orbitals into an enlarged-left set [0, m) and an
enlarged-right set [m, L), every monomial of

    H = sum h_pq a+_ps a_qs + 1/2 sum V_pqrs a+_ps a+_rt a_st a_qs

splits into a left factor and a right factor.  Reordering so that all left
operators stand before all right ones costs (-1)^(number of right operators
that had to pass a left operator).  The product then acts on |l>|r> as
(-1)^{N(l) * parity(right factor)} (L-factor|l>) (R-factor|r>), the sign rule
of the operator-sum matvec.

Monomials are grouped as:
  * all-left -> H_L (x) 1, all-right -> 1 (x) H_R;
  * one or two left operators -> that left monomial (x) (sum of right parts);
  * three left operators, one right operator -> (sum of left parts) (x) that
    right operator.
Every operator is built as an exact sparse matrix on the block's own Fock
space (Jordan-Wigner inside the block) and projected on the kept basis:
block = U_out^T M U_in.  Nothing here is renormalised step by step, so the
pairs are exactly P^T H P for P = U_L (x) U_R.
"""
from __future__ import annotations

from itertools import product

import numpy as np

from .fock import FockSpace


def _split(factors, m):
    left = [f for f in factors if f[1] < m]
    right = [(d, i - m, s) for (d, i, s) in factors if i >= m]
    inv = 0
    seen_right = 0
    for f in factors:
        if f[1] >= m:
            seen_right += 1
        else:
            inv += seen_right
    return tuple(left), tuple(right), (-1.0 if inv % 2 else 1.0)


def _dq(factors):
    dn = ds = 0
    for (dag, _i, s) in factors:
        sgn = 1 if dag else -1
        dn += sgn
        ds += sgn * (1 if s == 0 else -1)
    return (dn, ds)


def hamiltonian_monomials(h, V, tol=0.0):
    n = h.shape[0]
    for p, q in product(range(n), repeat=2):
        if abs(h[p, q]) > tol:
            for s in (0, 1):
                yield h[p, q], ((1, p, s), (0, q, s))
    for p, q, r, s_ in product(range(n), repeat=4):
        v = V[p, q, r, s_]
        if abs(v) > tol:
            for s, t in product((0, 1), repeat=2):
                yield 0.5 * v, ((1, p, s), (1, r, t), (0, s_, t), (0, q, s))


class _Basis:
    """Kept basis of one block: per (N, 2Sz) sector, an isometry from the
    block's Fock states of that sector (increasing index) to kept states."""

    def __init__(self, fs: FockSpace, iso=None):
        self.fs = fs
        qns = sorted({tuple(q) for q in fs.qn.tolist()})
        self.sectors = []
        for q in qns:
            states = fs.sector(*q)
            U = np.eye(len(states)) if iso is None else iso.get(q)
            if U is None or U.shape[1] == 0:
                continue
            self.sectors.append((q, states, U))
        self.qn = np.array([s[0] for s in self.sectors], dtype=np.int32).reshape(-1, 2)
        self.dim = np.array([s[2].shape[1] for s in self.sectors], dtype=np.int64)
        self.index = {s[0]: k for k, s in enumerate(self.sectors)}


def physical_problem(h, V, m, n_a, n_b, iso_left=None, iso_right=None):
    """Operator-pair problem for the cut after orbital m-1 at total
    (N, 2Sz) = (n_a+n_b, n_a-n_b).  Returns a synth.problem.Problem with
    psi = 0 (callers supply psi).  iso_left/iso_right map a sector (N, 2Sz)
    to an isometry (Fock states of that sector -> kept states); None keeps
    every Fock state."""
    import torch

    from synth.problem import Problem, Term

    L = h.shape[0]
    fsL, fsR = FockSpace(m), FockSpace(L - m)
    BL, BR = _Basis(fsL, iso_left), _Basis(fsR, iso_right)
    Q = np.array([n_a + n_b, n_a - n_b], dtype=np.int32)

    HL = None
    HR = None
    by_left = {}    # left monomial -> accumulated right operator
    by_right = {}   # right monomial -> accumulated left operator
    cacheL, cacheR = {}, {}

    def opL(f):
        if f not in cacheL:
            cacheL[f] = fsL.op(f)
        return cacheL[f]

    def opR(f):
        if f not in cacheR:
            cacheR[f] = fsR.op(f)
        return cacheR[f]

    for coeff, factors in hamiltonian_monomials(h, V):
        lf, rf, sgn = _split(factors, m)
        c = coeff * sgn
        if not rf:
            HL = c * opL(lf) if HL is None else HL + c * opL(lf)
        elif not lf:
            HR = c * opR(rf) if HR is None else HR + c * opR(rf)
        elif len(lf) <= 2:
            by_left[lf] = c * opR(rf) if lf not in by_left else by_left[lf] + c * opR(rf)
        else:
            by_right[rf] = c * opL(lf) if rf not in by_right else by_right[rf] + c * opL(lf)

    pairs = []  # (dq, odd, one_sided, Lmat or None, Rmat or None)
    if HL is not None:
        pairs.append(((0, 0), 0, 1, HL, None))
    if HR is not None:
        pairs.append(((0, 0), 0, 2, None, HR))
    for lf in sorted(by_left):
        # the right part carries 2-len(lf) or 4-len(lf) factors: same parity as lf
        pairs.append((_dq(lf), len(lf) % 2, 0, opL(lf), by_left[lf]))
    for rf in sorted(by_right):
        dn, ds = _dq(rf)  # shift of the right operator; the left side moves oppositely
        pairs.append(((-dn, -ds), len(rf) % 2, 0, by_right[rf], opR(rf)))

    def project(B, M, q_in, dq, sign):
        k_in = B.index.get(q_in)
        q_out = (q_in[0] + sign * dq[0], q_in[1] + sign * dq[1])
        k_out = B.index.get(q_out)
        if k_in is None or k_out is None:
            return None
        _, s_in, U_in = B.sectors[k_in]
        _, s_out, U_out = B.sectors[k_out]
        return U_out.T @ (M[s_out][:, s_in].toarray() @ U_in)

    lpool, rpool, terms = [], [], []
    loff_tot = roff_tot = 0
    for (dq, odd, one, ML, MR) in pairs:
        left_off = None if one == 2 else np.full(len(BL.dim), -1, dtype=np.int64)
        right_off = None if one == 1 else np.full(len(BR.dim), -1, dtype=np.int64)
        if ML is not None:
            for a, q in enumerate(BL.qn.tolist()):
                blk = project(BL, ML, tuple(q), dq, +1)
                if blk is not None and blk.size:
                    left_off[a] = loff_tot
                    lpool.append(blk.ravel())
                    loff_tot += blk.size
        if MR is not None:
            for c, r in enumerate(BR.qn.tolist()):
                blk = project(BR, MR, tuple(r), dq, -1)
                if blk is not None and blk.size:
                    right_off[c] = roff_tot
                    rpool.append(blk.ravel())
                    roff_tot += blk.size
        terms.append(Term(dq=tuple(dq), odd=odd, hc=0, one_sided=one, coeff=1.0,
                          left_off=left_off, right_off=right_off, group="phys"))
    lp = torch.from_numpy(np.concatenate(lpool) if lpool else np.zeros(1))
    rp = torch.from_numpy(np.concatenate(rpool) if rpool else np.zeros(1))
    prob = Problem(BL.qn, BL.dim, BR.qn, BR.dim, Q, terms, lp, rp, torch.zeros(0, dtype=torch.float64),
                   meta=dict(kind="physical", m=m, L=L))
    prob.bases = (BL, BR)
    return prob


def embedding(prob, states):
    """Dense P mapping psi-layout coordinates into a list of full Fock states.

    `states` holds full-space basis indices x = x_L + 2^{2m} x_R (e.g. the FCI
    sector basis); column k of P is the product basis vector U_L[:, i] (x)
    U_R[:, j] of psi entry k, so H_eff = P^T H P.
    """
    BL, BR = prob.bases
    m = BL.fs.n_orb
    row = {int(x): k for k, x in enumerate(np.asarray(states).tolist())}
    ridx = {tuple(r): k for k, r in enumerate(np.asarray(prob.Rq).tolist())}
    cols = []
    for a, q in enumerate(np.asarray(prob.Lq).tolist()):
        c = ridx.get((int(prob.Q[0]) - q[0], int(prob.Q[1]) - q[1]))
        if c is None:
            continue
        _, sL, UL = BL.sectors[a]
        _, sR, UR = BR.sectors[c]
        xs = (sL[:, None] + (sR[None, :] << (2 * m))).ravel()
        rows = np.array([row[int(x)] for x in xs])
        for i in range(UL.shape[1]):
            for j in range(UR.shape[1]):
                col = np.zeros(len(row))
                col[rows] = np.outer(UL[:, i], UR[:, j]).ravel()
                cols.append(col)
    return np.stack(cols, axis=1)

"""Seeded synthetic two-site effective-Hamiltonian problems.

Input construction only (no effective-Hamiltonian arithmetic): sector
tables, the list of operator-pair terms with their quantum-number shifts,
operator block values and the wavefunction.  The oracle and the HIP path
both consume exactly these arrays.

Term classes follow the normal/complementary operator split of ab initio
DMRG (the paper's Hamiltonian is the quantum-chemistry H of the Numerical
procedure section; the split itself is textbook DMRG): with k_L orbitals in
the enlarged left block and k_R in the enlarged right block,

  group     left op        right op    dq=(dN,d2Sz) odd hc  count
  HL        H_L            1           (0,0)        0   0   1
  HR        1              H_R         (0,0)        0   0   1
  CS_a/b    a+_{i,s}       S_{i,s}     (1,+-1)      1   1   k_L each
  SA_a/b    S_{j,s}        a_{j,s}     (1,+-1)      1   1   k_R each
  AP_aa/bb  a+_i a+_k      P           (2,+-2)      0   1   C(k_L,2) each
  AP_ab     a+_ia a+_kb    P           (2,0)        0   1   k_L^2
  BQ_diag   a+_is a_is     Q           (0,0)        0   0   2 k_L  (symmetric)
  BQ_off    a+_is a_js     Q           (0,0)        0   1   2 C(k_L,2)
  BQ_flip   a+_ia a_jb     Q           (0,2)        0   1   k_L^2

Values are calibration choices, not physics: H_L/H_R blocks are
diag(sorted 3|N(0,1)|) plus a symmetric N(0,1)/sqrt(2d) perturbation; two
sided blocks are i.i.d. N(0,1)/sqrt(d_in); BQ_diag blocks are symmetrised;
one-sided terms have coefficient 1 and two-sided terms 1/sqrt(n), n the
number of two-sided terms counting hermitian-conjugate partners; psi is
i.i.d. N(0,1) on every allowed block, normalised to 1.

Pool layout.  Operators of one group share one block layout, so each group
is a contiguous [n_ops, op_size] slab of its pool; inside one operator the
blocks follow the input-sector order.  A block is stored only when the
matvec can use it: input and output wavefunction blocks both exist.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from math import comb, sqrt

import numpy as np
import torch

from .sectors import bond_sectors

# (name, side-of-normal-op, dq, odd, hc, one_sided, symmetric)
GROUPS = (
    ("HL", "L", (0, 0), 0, 0, 1, True),
    ("HR", "R", (0, 0), 0, 0, 2, True),
    ("CS_a", "L", (1, 1), 1, 1, 0, False),
    ("CS_b", "L", (1, -1), 1, 1, 0, False),
    ("SA_a", "R", (1, 1), 1, 1, 0, False),
    ("SA_b", "R", (1, -1), 1, 1, 0, False),
    ("AP_aa", "L", (2, 2), 0, 1, 0, False),
    ("AP_bb", "L", (2, -2), 0, 1, 0, False),
    ("AP_ab", "L", (2, 0), 0, 1, 0, False),
    ("BQ_diag", "L", (0, 0), 0, 0, 0, True),
    ("BQ_off", "L", (0, 0), 0, 1, 0, False),
    ("BQ_flip", "L", (0, 2), 0, 1, 0, False),
)


def group_counts(kL: int, kR: int):
    c2 = comb(kL, 2)
    return {
        "HL": 1, "HR": 1,
        "CS_a": kL, "CS_b": kL, "SA_a": kR, "SA_b": kR,
        "AP_aa": c2, "AP_bb": c2, "AP_ab": kL * kL,
        "BQ_diag": 2 * kL, "BQ_off": 2 * c2, "BQ_flip": kL * kL,
    }


@dataclass
class Term:
    dq: tuple
    odd: int
    hc: int
    one_sided: int
    coeff: float
    left_off: np.ndarray | None   # int64[nL]: offset of O^L[q+dq, q] in left_pool, or -1
    right_off: np.ndarray | None  # int64[nR]: offset of O^R[r-dq, r] in right_pool, or -1
    group: str = ""


@dataclass
class Problem:
    Lq: np.ndarray   # int32[nL, 2]  (N, 2Sz) of enlarged-left sectors
    Ld: np.ndarray   # int64[nL]
    Rq: np.ndarray   # int32[nR, 2]
    Rd: np.ndarray   # int64[nR]
    Q: np.ndarray    # int32[2]
    terms: list
    left_pool: torch.Tensor
    right_pool: torch.Tensor
    psi: torch.Tensor
    meta: dict = field(default_factory=dict)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.Lq, self.Ld, self.Rq, self.Rd, self.Q):
            h.update(np.ascontiguousarray(a).tobytes())
        for t in self.terms:
            h.update(np.array([*t.dq, t.odd, t.hc, t.one_sided], dtype=np.int64).tobytes())
            h.update(np.float64(t.coeff).tobytes())
            for o in (t.left_off, t.right_off):
                if o is not None:
                    h.update(o.tobytes())
        for x in (self.left_pool, self.right_pool, self.psi):
            h.update(x.detach().cpu().numpy().tobytes())
        return h.hexdigest()


def _index(qn):
    return {tuple(q): i for i, q in enumerate(np.asarray(qn).tolist())}


def _useful_blocks(Lq, Ld, Rq, Rd, Q, dq):
    """Input sectors a (left) whose block O^L[q_a+dq, q_a] can contribute.

    Returns a list of (a, b, c, e): left in/out sector, right in/out sector.
    """
    li, ri = _index(Lq), _index(Rq)
    out = []
    for a, q in enumerate(Lq.tolist()):
        b = li.get((q[0] + dq[0], q[1] + dq[1]))
        c = ri.get((int(Q[0]) - q[0], int(Q[1]) - q[1]))
        if b is None or c is None:
            continue
        r = Rq[c].tolist()
        e = ri.get((r[0] - dq[0], r[1] - dq[1]))
        if e is None:
            continue
        out.append((a, b, c, e))
    return out


def psi_layout(Lq, Ld, Rq, Rd, Q):
    """Blocks (a, c, offset) of psi: left sector a, right sector c = Q - q_a."""
    ri = _index(Rq)
    blocks, off = [], 0
    for a, q in enumerate(Lq.tolist()):
        c = ri.get((int(Q[0]) - q[0], int(Q[1]) - q[1]))
        if c is None:
            continue
        blocks.append((a, c, off))
        off += int(Ld[a]) * int(Rd[c])
    return blocks, off


def _cap_counts(counts, sizes, budget_bytes):
    """Uniform cap of the two-sided groups so the pools fit a byte budget."""
    if budget_bytes is None:
        return dict(counts)
    fixed = sum(counts[g] * sizes[g] for g in ("HL", "HR")) * 8
    var = sum(counts[g] * sizes[g] for g in counts if g not in ("HL", "HR")) * 8
    f = min(1.0, max(0.0, (budget_bytes - fixed) / max(var, 1)))
    return {g: (n if g in ("HL", "HR") else max(1, int(n * f))) for g, n in counts.items()}


def make_problem(L: int, n_elec: int, two_sz: int, D: int, seed: int,
                 device="cpu", pool_budget_bytes=None, max_pairs_per_group=None,
                 sectors=None):
    """Build a seeded synthetic problem.

    pool_budget_bytes caps the two-sided groups uniformly so that both
    operator pools together stay within the budget (term count capped, block
    shapes untouched).  max_pairs_per_group caps each group's stored pairs
    (for small test problems).  `sectors` may pass explicit
    (Lq, Ld, Rq, Rd, Q) tables instead of the binomial rule.
    """
    if sectors is None:
        Lq, Ld, Rq, Rd, Q = bond_sectors(L, n_elec, two_sz, D)
    else:
        Lq, Ld, Rq, Rd, Q = (np.asarray(x) for x in sectors)
        Lq = Lq.astype(np.int32).reshape(-1, 2)
        Rq = Rq.astype(np.int32).reshape(-1, 2)
        Ld = Ld.astype(np.int64)
        Rd = Rd.astype(np.int64)
        Q = Q.astype(np.int32)
    kL = L // 2
    kR = L - kL
    counts = group_counts(kL, kR)
    nL, nR = len(Ld), len(Rd)

    # per-group block lists and per-op sizes
    blocks = {}
    lsize, rsize = {}, {}
    for (g, _side, dq, _odd, _hc, one, _sym) in GROUPS:
        ub = _useful_blocks(Lq, Ld, Rq, Rd, Q, dq)
        blocks[g] = ub
        lsize[g] = sum(int(Ld[b]) * int(Ld[a]) for (a, b, c, e) in ub) if one != 2 else 0
        rsize[g] = sum(int(Rd[e]) * int(Rd[c]) for (a, b, c, e) in ub) if one != 1 else 0
    sizes = {g: lsize[g] + rsize[g] for g in counts}
    if max_pairs_per_group is not None:
        counts = {g: (n if g in ("HL", "HR") else min(n, max_pairs_per_group)) for g, n in counts.items()}
    counts = _cap_counts(counts, sizes, pool_budget_bytes)

    n_two = sum(counts[g] * (2 if hc else 1) for (g, _s, _d, _o, hc, one, _y) in GROUPS if one == 0)
    c_two = 1.0 / sqrt(max(n_two, 1))

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.float64

    # ---- pools
    ltot = sum(counts[g] * lsize[g] for g in counts)
    rtot = sum(counts[g] * rsize[g] for g in counts)
    left_pool = torch.empty(max(ltot, 1), dtype=dt, device=device)
    right_pool = torch.empty(max(rtot, 1), dtype=dt, device=device)

    terms = []
    lbase = rbase = 0
    for (g, _side, dq, odd, hc, one, sym) in GROUPS:
        n = counts[g]
        ub = blocks[g]
        for side in ("L", "R"):
            if (side == "L" and one == 2) or (side == "R" and one == 1):
                continue
            size = lsize[g] if side == "L" else rsize[g]
            pool = left_pool if side == "L" else right_pool
            base = lbase if side == "L" else rbase
            slab = pool[base:base + n * size].view(n, size) if size else None
            if slab is not None:
                slab.normal_(generator=gen)
            off = 0
            for (a, b, c, e) in ub:
                rows, cols = (int(Ld[b]), int(Ld[a])) if side == "L" else (int(Rd[e]), int(Rd[c]))
                blk = slab[:, off:off + rows * cols].view(n, rows, cols)
                if one:
                    # Hamiltonian-like diagonal block of a one-sided term
                    z = torch.randn(n, rows, generator=gen, dtype=dt, device=device)
                    diag = torch.sort(3.0 * z.abs(), dim=1).values
                    blk.mul_(1.0 / sqrt(2.0 * rows))
                    up = torch.triu(blk)
                    blk.copy_(up + torch.triu(blk, 1).transpose(1, 2))
                    blk.diagonal(dim1=1, dim2=2).add_(diag)
                elif sym:
                    blk.mul_(1.0 / sqrt(cols))
                    blk.copy_((blk + blk.transpose(1, 2)) * (1.0 / sqrt(2.0)))
                else:
                    blk.mul_(1.0 / sqrt(cols))
                off += rows * cols
        # offsets of every op of this group
        loff_local = np.full(nL, -1, dtype=np.int64)
        roff_local = np.full(nR, -1, dtype=np.int64)
        lo = ro = 0
        for (a, b, c, e) in ub:
            if one != 2:
                loff_local[a] = lo
                lo += int(Ld[b]) * int(Ld[a])
            if one != 1:
                roff_local[c] = ro
                ro += int(Rd[e]) * int(Rd[c])
        for i in range(n):
            lo_arr = None if one == 2 else np.where(loff_local >= 0, loff_local + lbase + i * lsize[g], -1)
            ro_arr = None if one == 1 else np.where(roff_local >= 0, roff_local + rbase + i * rsize[g], -1)
            coeff = 1.0 if one else c_two
            terms.append(Term(dq=tuple(dq), odd=odd, hc=hc, one_sided=one, coeff=coeff,
                              left_off=lo_arr, right_off=ro_arr, group=g))
        lbase += n * lsize[g]
        rbase += n * rsize[g]

    _, total = psi_layout(Lq, Ld, Rq, Rd, Q)
    psi = torch.randn(total, generator=gen, dtype=dt, device=device)
    psi /= torch.linalg.vector_norm(psi)
    meta = dict(L=L, n_elec=n_elec, two_sz=two_sz, D=D, seed=seed, counts=counts,
                n_terms=sum(1 + t.hc for t in terms), n_pairs=len(terms),
                pool_bytes=8 * (ltot + rtot), psi_len=total)
    return Problem(Lq, Ld, Rq, Rd, Q, terms, left_pool, right_pool, psi, meta)


# Named workloads (seeds 1001..1005).  The three large ones take their shapes
# from the active spaces of the paper's benchmarks (L orbitals, N electrons,
# 2Sz, U(1) bond dimension D).
WORKLOADS = {
    "l24_d1024": dict(L=24, n_elec=24, two_sz=0, D=1024, seed=1002),
    "cas63_58_d4096": dict(L=58, n_elec=63, two_sz=1, D=4096, seed=1004),
    "cas113_76_d8192": dict(L=76, n_elec=113, two_sz=3, D=8192, seed=1005),
}

"""Seeded synthetic SU(2) spin-adapted two-site problems.

Input construction only (no effective-Hamiltonian arithmetic): multiplet
sector tables (N, 2j) with multiplet counts, operator-pair terms with their
spin rank and particle-number shift, random reduced blocks and the reduced
wavefunction.  Electrons carry spin 1/2, so N electrons couple to integer j
for even N and half-integer j for odd N; every sector respects that.

Term classes (spin-adapted counterparts of synth.problem's groups):

  group   left op         right op   2k  dN  odd hc  one_sided
  HL      H_L             1          0   0   0   0   1
  HR      1               H_R        0   0   0   0   2
  CS      a+_i            S_i        1   1   1   1   0
  SA      S_j             a_j        1   1   1   1   0
  AP0     [a+ a+]^0       P^0        0   2   0   1   0
  AP1     [a+ a+]^1       P^1        2   2   0   1   0
  BQ0     [a+ a]^0        Q^0        0   0   0   0   0   (symmetric blocks)
  BQ1     [a+ a]^1        Q^1        2   0   0   1   0

A reduced block O[(N', j'), (N, j)] is stored for every pair of sectors with
N' = N + dN and |j - k| <= j' <= j + k; values i.i.d. N(0,1)/sqrt(d_in)
(one-sided blocks: sorted 3|N(0,1)| diagonal plus a symmetric perturbation);
two-sided coefficients 1/sqrt(n), n the two-sided terms counting hc.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import sqrt

import numpy as np
import torch

# (name, 2k, dN, odd, hc, one_sided, symmetric)
GROUPS_SU2 = (
    ("HL", 0, 0, 0, 0, 1, True),
    ("HR", 0, 0, 0, 0, 2, True),
    ("CS", 1, 1, 1, 1, 0, False),
    ("SA", 1, 1, 1, 1, 0, False),
    ("AP0", 0, 2, 0, 1, 0, False),
    ("AP1", 2, 2, 0, 1, 0, False),
    ("BQ0", 0, 0, 0, 0, 0, True),
    ("BQ1", 2, 0, 0, 1, 0, False),
)


@dataclass
class TermSU2:
    two_k: int
    dn: int
    odd: int
    hc: int
    one_sided: int
    coeff: float
    left_blocks: np.ndarray | None   # int64[n, 3]: output sector, input sector, pool offset
    right_blocks: np.ndarray | None
    group: str = ""


@dataclass
class ProblemSU2:
    Lq: np.ndarray   # int32[nL, 2]: (N, 2j)
    Ld: np.ndarray   # int64[nL]: multiplets per sector
    Rq: np.ndarray
    Rd: np.ndarray
    Q: np.ndarray    # int32[2]: (N, 2S)
    terms: list
    left_pool: torch.Tensor
    right_pool: torch.Tensor
    psi: torch.Tensor
    meta: dict = field(default_factory=dict)


def small_sectors(rng, n_lo, n_hi, tj_max, dmax):
    """Every (N, 2j) with n_lo <= N <= n_hi, 2j <= min(N, tj_max) and the
    electron parity rule; multiplet counts uniform in 1..dmax."""
    q, d = [], []
    for N in range(n_lo, n_hi + 1):
        for tj in range(N % 2, min(N, tj_max) + 1, 2):
            q.append((N, tj))
            d.append(int(rng.integers(1, dmax + 1)))
    return np.array(q, dtype=np.int32), np.array(d, dtype=np.int64)


def _allowed(q_in, q_out, dn, tk):
    dN = int(q_out[0]) - int(q_in[0])
    tj, tj2 = int(q_in[1]), int(q_out[1])
    return dN == dn and abs(tj - tk) <= tj2 <= tj + tk and (tj + tk + tj2) % 2 == 0


def _psi_blocks(Lq, Rq, Q):
    out = []
    for a in range(len(Lq)):
        for c in range(len(Rq)):
            if int(Lq[a][0]) + int(Rq[c][0]) != int(Q[0]):
                continue
            ta, tc, tS = int(Lq[a][1]), int(Rq[c][1]), int(Q[1])
            if abs(ta - tc) <= tS <= ta + tc and (ta + tc + tS) % 2 == 0:
                out.append((a, c))
    return out


# ---------------------------------------------------------------------------
# Multiplet sector tables of the middle bond (the spin-adapted counterpart
# of synth.sectors).  Per block of k orbitals the U(1) rule weighs (n_up,
# n_dn) by binomial(10, 1/2) occupations centred at floor(N/2 k/L + 1/2)
# for both spins; the states of N electrons with 2Sz = 2m then weigh
# D(N, m), symmetric in m and falling with |m|, and the multiplets of spin
# j weigh D(N, j) - D(N, j + 1).  Sectors with no partner on the other side
# are dropped and the weights scaled to D multiplets (largest remainder).
# The enlarged blocks add one site: multiplets (N, j) x {(0, 0), (1, 1/2),
# (2, 0)}, spin 1/2 coupling j to j -+ 1/2.

def _block_multiplets(k, L, n_elec):
    from .sectors import _spin_weights
    import math
    c = int(math.floor(n_elec / 2.0 * k / L + 0.5))
    w = _spin_weights(c, k)
    states = {}
    for na, wa in w.items():
        for nb, wb in w.items():
            key = (na + nb, na - nb)
            states[key] = states.get(key, 0) + wa * wb
    mult = {}
    for (N, tm), v in states.items():
        if tm < 0:
            continue
        nxt = states.get((N, tm + 2), 0)
        if v - nxt > 0:
            mult[(N, tm)] = v - nxt
    return mult


def _couples(tj1, tj2, tS):
    return abs(tj1 - tj2) <= tS <= tj1 + tj2 and (tj1 + tj2 + tS) % 2 == 0


def _enlarge_su2(block):
    acc = {}
    for (N, tj), d in block.items():
        for (sN, stj) in ((0, 0), (1, 1), (2, 0)):
            for tj2 in range(abs(tj - stj), tj + stj + 1, 2):
                key = (N + sN, tj2)
                acc[key] = acc.get(key, 0) + d
    keys = sorted(acc)
    return (np.array(keys, dtype=np.int32).reshape(-1, 2), np.array([acc[k] for k in keys], dtype=np.int64))


def bond_sectors_su2(L, n_elec, two_s, D):
    """Enlarged left/right multiplet tables and Q = (N, 2S) at the middle bond."""
    from .sectors import _largest_remainder
    assert (n_elec + two_s) % 2 == 0
    kl = L // 2 - 1
    kr = L - kl - 2
    left, right = _block_multiplets(kl, L, n_elec), _block_multiplets(kr, L, n_elec)

    def partner(s, others):
        # an enlarged pair (each block plus its site) can reach (n_elec, S)
        N, tj = s
        for (N2, tj2) in others:
            if 0 <= n_elec - N - N2 <= 4:
                for a in (tj - 1, tj, tj + 1):
                    for b in (tj2 - 1, tj2, tj2 + 1):
                        if a >= 0 and b >= 0 and _couples(a, b, two_s):
                            return True
        return False

    while True:
        kl_ = {s: w for s, w in left.items() if partner(s, right)}
        kr_ = {s: w for s, w in right.items() if partner(s, kl_)}
        if len(kl_) == len(left) and len(kr_) == len(right):
            break
        left, right = kl_, kr_
    out = []
    for side in (left, right):
        keys = sorted(side)
        dims = _largest_remainder([side[k] for k in keys], D)
        out.append({k: int(d) for k, d in zip(keys, dims) if d > 0})
    Lq, Ld = _enlarge_su2(out[0])
    Rq, Rd = _enlarge_su2(out[1])
    return Lq, Ld, Rq, Rd, np.array([n_elec, two_s], dtype=np.int32)


def _useful(q, other_q, pblocks_of, dn, tk):
    """Stored blocks (out, in) of one side whose input and output reduced
    wavefunction blocks both exist with right partners the other operator
    (same rank, opposite shift) can connect."""
    rows = []
    n = len(q)
    for a in range(n):
        if a not in pblocks_of:
            continue
        for a2 in range(n):
            if a2 not in pblocks_of or not _allowed(q[a], q[a2], dn, tk):
                continue
            ok = False
            for c in pblocks_of[a]:
                for c2 in pblocks_of[a2]:
                    tjc, tjc2 = int(other_q[c][1]), int(other_q[c2][1])
                    if abs(tjc - tk) <= tjc2 <= tjc + tk and (tjc + tk + tjc2) % 2 == 0:
                        ok = True
                        break
                if ok:
                    break
            if ok:
                rows.append((a2, a))
    return rows


def make_problem_su2(Lq, Ld, Rq, Rd, Q, seed, counts=None, device="cpu", pairs=2, pool_budget_bytes=None):
    """Terms of every group (counts: {group: n}; default `pairs` each and one
    for HL / HR), a block for every sector pair the wavefunction can use,
    seeded values (one torch generator, group by group), capped uniformly
    in term count to pool_budget_bytes."""
    Lq = np.asarray(Lq, dtype=np.int32).reshape(-1, 2)
    Rq = np.asarray(Rq, dtype=np.int32).reshape(-1, 2)
    Ld = np.asarray(Ld, dtype=np.int64)
    Rd = np.asarray(Rd, dtype=np.int64)
    Q = np.asarray(Q, dtype=np.int32).reshape(2)
    tS = int(Q[1])
    pblocks = _psi_blocks(Lq, Rq, Q)
    lpart, rpart = {}, {}
    for a, c in pblocks:
        lpart.setdefault(a, []).append(c)
        rpart.setdefault(c, []).append(a)
    counts = dict(counts or {g[0]: (1 if g[5] else pairs) for g in GROUPS_SU2})
    layouts = {}
    for (g, tk, dn, odd, hc, one, sym) in GROUPS_SU2:
        if one == 1:
            lrows = [(a, a) for a in sorted(lpart)]
            rrows = []
        elif one == 2:
            lrows = []
            rrows = [(c, c) for c in sorted(rpart)]
        else:
            lrows = _useful(Lq, Rq, lpart, dn, tk)
            rrows = _useful(Rq, Lq, rpart, -dn, tk)
        lsz = sum(int(Ld[o] * Ld[i]) for o, i in lrows)
        rsz = sum(int(Rd[o] * Rd[i]) for o, i in rrows)
        layouts[g] = (lrows, rrows, lsz, rsz)
    if pool_budget_bytes is not None:
        fixed = sum(counts.get(g[0], 0) * (layouts[g[0]][2] + layouts[g[0]][3]) for g in GROUPS_SU2 if g[5]) * 8
        var = sum(counts.get(g[0], 0) * (layouts[g[0]][2] + layouts[g[0]][3]) for g in GROUPS_SU2 if not g[5]) * 8
        f = min(1.0, max(0.0, (pool_budget_bytes - fixed) / max(var, 1)))
        counts = {g: (n if g in ("HL", "HR") else max(1, int(n * f))) for g, n in counts.items()}
    n_two = sum(counts.get(g[0], 0) * (2 if g[4] else 1) for g in GROUPS_SU2 if g[5] == 0)
    c_two = 1.0 / sqrt(max(n_two, 1))
    dt = torch.float64
    ltot = sum(counts.get(g, 0) * layouts[g][2] for g in layouts)
    rtot = sum(counts.get(g, 0) * layouts[g][3] for g in layouts)
    left_pool = torch.empty(max(ltot, 1), dtype=dt, device=device)
    right_pool = torch.empty(max(rtot, 1), dtype=dt, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    terms = []
    lbase = rbase = 0
    for (g, tk, dn, odd, hc, one, sym) in GROUPS_SU2:
        n = counts.get(g, 0)
        if n == 0:
            continue
        lrows, rrows, lsz, rsz = layouts[g]
        tabs = []
        for side, rows, size, q, d, pool, base in (("L", lrows, lsz, Lq, Ld, left_pool, lbase),
                                                   ("R", rrows, rsz, Rq, Rd, right_pool, rbase)):
            if (side == "L" and one == 2) or (side == "R" and one == 1):
                tabs.append(None)
                continue
            slab = pool[base:base + n * size].view(n, size) if size else None
            if slab is not None:
                slab.normal_(generator=gen)
            off = 0
            local = []
            for (o, i) in rows:
                r, cdim = int(d[o]), int(d[i])
                blk = slab[:, off:off + r * cdim].view(n, r, cdim)
                if one:
                    z = torch.randn(n, r, generator=gen, dtype=dt, device=device)
                    diag = torch.sort(3.0 * z.abs(), dim=1).values
                    blk.mul_(1.0 / sqrt(2.0 * r))
                    blk.copy_(torch.triu(blk) + torch.triu(blk, 1).transpose(1, 2))
                    blk.diagonal(dim1=1, dim2=2).add_(diag)
                elif sym and o == i:
                    blk.mul_(1.0 / sqrt(cdim))
                    blk.copy_((blk + blk.transpose(1, 2)) * (1.0 / sqrt(2.0)))
                else:
                    blk.mul_(1.0 / sqrt(cdim))
                local.append((o, i, off))
                off += r * cdim
            tabs.append((np.array(local, dtype=np.int64).reshape(-1, 3), base, size))
        for t_i in range(n):
            lb = rb = None
            if tabs[0] is not None:
                arr, base, size = tabs[0]
                lb = arr.copy()
                lb[:, 2] += base + t_i * size
            if tabs[1] is not None:
                arr, base, size = tabs[1]
                rb = arr.copy()
                rb[:, 2] += base + t_i * size
            terms.append(TermSU2(two_k=tk, dn=dn, odd=odd, hc=hc, one_sided=one,
                                 coeff=1.0 if one else c_two, left_blocks=lb, right_blocks=rb, group=g))
        lbase += n * lsz
        rbase += n * rsz
    total = sum(int(Ld[a] * Rd[c]) for a, c in pblocks)
    psi = torch.randn(total, generator=gen, dtype=dt, device=device)
    psi /= torch.linalg.vector_norm(psi)
    meta = dict(seed=seed, counts=counts, n_terms=sum(1 + t.hc for t in terms), n_pairs=len(terms),
                psi_len=total, pool_bytes=8 * (ltot + rtot))
    return ProblemSU2(Lq, Ld, Rq, Rd, Q, terms, left_pool, right_pool, psi, meta)


def tiny_su2(seed=1, n_lo=1, n_hi=4, tj_max=3, dmax=3, N=6, two_s=1, pairs=2, device="cpu"):
    """A small problem: left and right sectors with n_lo..n_hi electrons and
    2j up to tj_max, total (N, 2S)."""
    rng = np.random.default_rng(seed + 7919)
    Lq, Ld = small_sectors(rng, n_lo, n_hi, tj_max, dmax)
    Rq, Rd = small_sectors(rng, n_lo, n_hi, tj_max, dmax)
    return make_problem_su2(Lq, Ld, Rq, Rd, (N, two_s), seed, device=device, pairs=pairs)


def group_counts_su2(kL, kR):
    """Operator pairs per group at the middle bond (k_L / k_R orbitals in
    the enlarged blocks)."""
    return {"HL": 1, "HR": 1, "CS": kL, "SA": kR, "AP0": kL * (kL + 1) // 2, "AP1": kL * (kL - 1) // 2,
            "BQ0": kL * (kL + 1) // 2, "BQ1": kL * (kL + 1) // 2}


WORKLOADS_SU2 = {
    "su2_cas63_58_d4096": dict(L=58, n_elec=63, two_s=1, D=4096, seed=2004),
    "su2_l24_d512": dict(L=24, n_elec=24, two_s=0, D=512, seed=2002),
}


def make_workload_su2(name, device="cpu", pool_budget_bytes=None):
    w = WORKLOADS_SU2[name]
    Lq, Ld, Rq, Rd, Q = bond_sectors_su2(w["L"], w["n_elec"], w["two_s"], w["D"])
    kL = w["L"] // 2
    kR = w["L"] - kL
    return make_problem_su2(Lq, Ld, Rq, Rd, Q, w["seed"], counts=group_counts_su2(kL, kR), device=device,
                            pool_budget_bytes=pool_budget_bytes)

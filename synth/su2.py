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


def make_problem_su2(Lq, Ld, Rq, Rd, Q, seed, counts=None, device="cpu", pairs=2):
    """Terms of every group (counts: {group: n}, default `pairs` each, one
    for HL / HR), blocks for every allowed sector pair the wavefunction can
    use, seeded values."""
    rng = np.random.default_rng(seed)
    Lq = np.asarray(Lq, dtype=np.int32).reshape(-1, 2)
    Rq = np.asarray(Rq, dtype=np.int32).reshape(-1, 2)
    Ld = np.asarray(Ld, dtype=np.int64)
    Rd = np.asarray(Rd, dtype=np.int64)
    Q = np.asarray(Q, dtype=np.int32).reshape(2)
    pblocks = _psi_blocks(Lq, Rq, Q)
    lin = {a for a, _ in pblocks}
    rin = {c for _, c in pblocks}
    counts = counts or {g[0]: (1 if g[5] else pairs) for g in GROUPS_SU2}
    n_two = sum(counts.get(g[0], 0) * (2 if g[4] else 1) for g in GROUPS_SU2 if g[5] == 0)
    c_two = 1.0 / sqrt(max(n_two, 1))
    lpool, rpool, terms = [], [], []
    lsize = rsize = 0

    def blocks_of(q, d, used, dn, tk, sym, one, pool, size):
        rows = []
        for a in range(len(q)):
            if a not in used:
                continue
            for a2 in range(len(q)):
                if a2 not in used or not _allowed(q[a], q[a2], dn, tk):
                    continue
                m = rng.standard_normal((int(d[a2]), int(d[a])))
                if one:
                    m = m / sqrt(2.0 * d[a])
                    m = np.triu(m) + np.triu(m, 1).T + np.diag(np.sort(3.0 * np.abs(rng.standard_normal(int(d[a])))))
                elif sym and a2 == a:
                    m = (m + m.T) / sqrt(2.0 * d[a])
                else:
                    m = m / sqrt(float(d[a]))
                rows.append((a2, a, size))
                pool.append(m.reshape(-1))
                size += m.size
        return np.array(rows, dtype=np.int64).reshape(-1, 3), size

    for (g, tk, dn, odd, hc, one, sym) in GROUPS_SU2:
        for _ in range(counts.get(g, 0)):
            lb = rb = None
            if one != 2:
                lb, lsize = blocks_of(Lq, Ld, lin, dn, tk, sym, one == 1, lpool, lsize)
            if one != 1:
                rb, rsize = blocks_of(Rq, Rd, rin, -dn, tk, sym, one == 2, rpool, rsize)
            terms.append(TermSU2(two_k=tk, dn=dn, odd=odd, hc=hc, one_sided=one,
                                 coeff=1.0 if one else c_two, left_blocks=lb, right_blocks=rb, group=g))
    total = sum(int(Ld[a] * Rd[c]) for a, c in pblocks)
    psi = rng.standard_normal(total)
    psi /= np.linalg.norm(psi)
    dt = torch.float64
    lp = torch.from_numpy(np.concatenate(lpool) if lpool else np.zeros(1)).to(device=device, dtype=dt)
    rp = torch.from_numpy(np.concatenate(rpool) if rpool else np.zeros(1)).to(device=device, dtype=dt)
    meta = dict(seed=seed, n_terms=sum(1 + t.hc for t in terms), n_pairs=len(terms), psi_len=total,
                pool_bytes=8 * (lsize + rsize))
    return ProblemSU2(Lq, Ld, Rq, Rd, Q, terms, lp, rp, torch.from_numpy(psi).to(device=device, dtype=dt), meta)


def tiny_su2(seed=1, n_lo=1, n_hi=4, tj_max=3, dmax=3, N=6, two_s=1, pairs=2, device="cpu"):
    """A small problem: left and right sectors with n_lo..n_hi electrons and
    2j up to tj_max, total (N, 2S)."""
    rng = np.random.default_rng(seed + 7919)
    Lq, Ld = small_sectors(rng, n_lo, n_hi, tj_max, dmax)
    Rq, Rd = small_sectors(rng, n_lo, n_hi, tj_max, dmax)
    return make_problem_su2(Lq, Ld, Rq, Rd, (N, two_s), seed, device=device, pairs=pairs)

"""Synthetic U(1)xU(1) sector tables for the two-site DMRG bond.

Input construction only: this module decides which (N, 2Sz) sectors the
left and right blocks carry and how many states each holds.  It contains
none of the effective-Hamiltonian arithmetic.

The paper quotes bond dimensions D for active spaces of M electrons in N
orbitals (Performance assessment section) but no sector tables, so the
sectors are synthetic:

* the middle bond splits L orbitals into a left block [0, L/2-2], the two
  dot sites L/2-1 and L/2, and a right block holding the rest;
* per block of k orbitals and per spin sigma, occupation n_sigma takes
  binomial(10, 1/2) weights centred at floor(N_sigma*k/L + 1/2) (centre +-5,
  clipped to [0, k]); the sector weight is the product over the two spins;
* sectors with no complement on the other side are dropped, the rest are
  scaled to D with largest-remainder rounding (ties by sector order) and
  empty sectors dropped;
* the enlarged left block is (left block) x (site L/2-1), the enlarged
  right block is (site L/2) x (right block); each carries the 4 site states
  |0>, |up>, |dn>, |updn> with (N, 2Sz) = (0,0), (1,1), (1,-1), (2,0).
"""
from __future__ import annotations

from math import comb, floor

import numpy as np

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _spin_weights(centre: int, k: int, width: int = 10):
    half = width // 2
    out = {}
    for n in range(centre - half, centre + half + 1):
        if 0 <= n <= k:
            out[n] = comb(width, n - centre + half)
    return out


def _candidates(k: int, L: int, n_a: int, n_b: int):
    ca = int(floor(n_a * k / L + 0.5))
    cb = int(floor(n_b * k / L + 0.5))
    wa = _spin_weights(ca, k)
    wb = _spin_weights(cb, k)
    return {(na, nb): wa[na] * wb[nb] for na in wa for nb in wb}


def _has_complement(s, others, n_a, n_b):
    na, nb = s
    for (ma, mb) in others:
        if 0 <= n_a - na - ma <= 2 and 0 <= n_b - nb - mb <= 2:
            return True
    return False


def _largest_remainder(weights, total):
    w = np.asarray(weights, dtype=np.float64)
    exact = w * total / w.sum()
    base = np.floor(exact).astype(np.int64)
    rem = exact - base
    short = int(total - base.sum())
    # ties broken by sector order: stable sort on -remainder
    order = np.argsort(-rem, kind="stable")
    base[order[:short]] += 1
    return base


def block_sectors(L: int, n_a: int, n_b: int, D: int):
    """Sectors of the left and right blocks at the middle bond.

    Returns two lists of ((N, 2Sz), dim) sorted by (N, 2Sz), one per block,
    with dims summing to D on each side.
    """
    k = L // 2 - 1
    left = _candidates(k, L, n_a, n_b)
    right = _candidates(L - k - 2, L, n_a, n_b)
    while True:
        keep_l = {s: w for s, w in left.items() if _has_complement(s, right, n_a, n_b)}
        keep_r = {s: w for s, w in right.items() if _has_complement(s, keep_l, n_a, n_b)}
        if len(keep_l) == len(left) and len(keep_r) == len(right):
            break
        left, right = keep_l, keep_r
    out = []
    for side in (left, right):
        keys = sorted(side, key=lambda s: (s[0] + s[1], s[0] - s[1]))
        dims = _largest_remainder([side[s] for s in keys], D)
        out.append({s: int(d) for s, d in zip(keys, dims) if d > 0})
    # dropping empty sectors may orphan sectors on the other side: repeat
    left, right = out
    while True:
        keep_l = {s: d for s, d in left.items() if _has_complement(s, right, n_a, n_b)}
        keep_r = {s: d for s, d in right.items() if _has_complement(s, keep_l, n_a, n_b)}
        if len(keep_l) == len(left) and len(keep_r) == len(right):
            break
        left, right = keep_l, keep_r

    def as_list(side):
        items = [((na + nb, na - nb), d) for (na, nb), d in side.items()]
        return sorted(items)

    return as_list(left), as_list(right)


def enlarge(block, site_first: bool):
    """Combine a block's sectors with the 4 states of one site.

    Returns (qn int32[n,2], dim int64[n]) sorted by (N, 2Sz).  The order of
    states inside an enlarged sector is irrelevant for synthetic operators.
    """
    acc = {}
    for (q, d) in block:
        for sq in SITE_QN:
            t = (q[0] + sq[0], q[1] + sq[1])
            acc[t] = acc.get(t, 0) + d
    keys = sorted(acc)
    qn = np.array(keys, dtype=np.int32).reshape(-1, 2)
    dim = np.array([acc[t] for t in keys], dtype=np.int64)
    return qn, dim


def bond_sectors(L: int, n_elec: int, two_sz: int, D: int):
    """Enlarged left/right sector tables and total quantum numbers Q.

    n_alpha = (N + 2Sz)/2, n_beta = (N - 2Sz)/2.
    """
    assert (n_elec + two_sz) % 2 == 0
    n_a = (n_elec + two_sz) // 2
    n_b = (n_elec - two_sz) // 2
    lb, rb = block_sectors(L, n_a, n_b, D)
    Lq, Ld = enlarge(lb, site_first=False)
    Rq, Rd = enlarge(rb, site_first=True)
    return Lq, Ld, Rq, Rd, np.array([n_elec, two_sz], dtype=np.int32)

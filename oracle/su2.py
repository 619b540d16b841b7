"""SU(2) spin-adapted two-site effective Hamiltonian, plain definition
(oracle; test infrastructure).

The paper's DMRG is spin adapted: its bond dimensions count SU(2) multiplets
(Introduction; Performance assessment section; the P450 section quotes
D = 4096 multiplets as about 11000 U(1) states).  It gives no formulas; this
module states the standard construction.

Sectors of an enlarged block are (N, 2j) with d multiplets each (every
multiplet holds 2j + 1 states).  An operator of spin rank k is stored by its
reduced blocks O[(N', j'), (N, j)] (d' x d) in the Wigner-Eckart convention

    <j' m' i'| T^k_q |j m i> = <j m; k q | j' m'> O[(N', j'), (N, j)][i', i],

with Clebsch-Gordan coefficients <j1 m1; j2 m2 | J M> (Condon-Shortley).  A
term of the two-site Hamiltonian is the scalar

    c * sum_q (-1)^(k - q) T_q (x) U_{-q}

(T on the left block, U on the right, k integer or half-integer; for k = 0
it is c T (x) U), times the fermionic sign (-1)^N(left input) when U changes
the particle number by an odd amount; one-sided terms are c T (x) 1 or
c 1 (x) U with k = 0.  The wavefunction of total (N, S) stores one reduced
block Psi[(a, c)] (d_a x d_c) for every left sector a and right sector c
with N_a + N_c = N and |j_a - j_c| <= S <= j_a + j_c; the full state is
sum Psi[a,c][i,j] |(j_a i, j_c j) S M>, the same for every M.

The reduced matvec multiplies each stored block pair by the weight

    W = <(j_a' j_c') S M| sum_q (-1)^(k-q) t_q (x) u_{-q} |(j_a j_c) S M>

of unit reduced operators, computed here from its definition: a sum over
magnetic quantum numbers of products of Clebsch-Gordan coefficients (M-
independent by the Wigner-Eckart theorem, which a pin checks).  A term with
hc = 1 also applies the transpose of each of its contributions (the
hermitian conjugate of a real symmetric-form term).

expand_to_u1 writes the same problem in the U(1) x U(1) (N, 2Sz) form of
oracle.heff, which applies it independently.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache
from math import factorial, sqrt

import numpy as np

# ---------------------------------------------------------------------------
# Clebsch-Gordan coefficients.  Arguments are doubled (tj = 2j, tm = 2m), so
# every spin is an integer here.


def _tri(a, b, c):
    """Triangle rule for doubled spins (and integer total)."""
    return abs(a - b) <= c <= a + b and (a + b + c) % 2 == 0


@lru_cache(maxsize=None)
def cg(tj1, tm1, tj2, tm2, tJ, tM):
    """<j1 m1; j2 m2 | J M> by Racah's closed formula, exact in rationals
    until the final square root."""
    if tm1 + tm2 != tM or not _tri(tj1, tj2, tJ):
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    f = lambda x: factorial(x // 2)  # noqa: E731  (x is even)
    pre = Fraction((tJ + 1) * f(tJ + tj1 - tj2) * f(tJ - tj1 + tj2) * f(tj1 + tj2 - tJ),
                   f(tj1 + tj2 + tJ + 2))
    pre *= (f(tJ + tM) * f(tJ - tM) * f(tj1 - tm1) * f(tj1 + tm1) * f(tj2 - tm2) * f(tj2 + tm2))
    s = Fraction(0)
    for k2 in range(0, tj1 + tj2 - tJ + 1, 2):
        args = (k2, tj1 + tj2 - tJ - k2, tj1 - tm1 - k2, tj2 + tm2 - k2, tJ - tj2 + tm1 + k2,
                tJ - tj1 - tm2 + k2)
        if min(args) < 0:
            continue
        den = 1
        for x in args:
            den *= f(x)
        s += Fraction((-1) ** (k2 // 2), den)
    return float(s) * sqrt(float(pre)) if s != 0 else 0.0


def weight(tja, tjc, tja2, tjc2, tk, tS, tM=None):
    """W of a two-sided term for unit reduced operators, from its definition
    (sum over magnetic quantum numbers at M; default M = S)."""
    tM = tS if tM is None else tM
    w = 0.0
    for tma in range(-tja, tja + 1, 2):
        tmc = tM - tma
        if abs(tmc) > tjc:
            continue
        cin = cg(tja, tma, tjc, tmc, tS, tM)
        if cin == 0.0:
            continue
        for tq in range(-tk, tk + 1, 2):
            tma2, tmc2 = tma + tq, tmc - tq
            if abs(tma2) > tja2 or abs(tmc2) > tjc2:
                continue
            cout = cg(tja2, tma2, tjc2, tmc2, tS, tM)
            if cout == 0.0:
                continue
            phase = -1.0 if ((tk - tq) // 2) % 2 else 1.0
            w += cout * cin * phase * cg(tja, tma, tk, tq, tja2, tma2) * cg(tjc, tmc, tk, -tq, tjc2, tmc2)
    return w


# ---------------------------------------------------------------------------
# Problem description: any object with the fields of synth.su2.ProblemSU2
# (Lq, Ld, Rq, Rd, Q = (N, 2S), terms, left_pool, right_pool, psi); each term
# has two_k, dn, odd, hc, one_sided, coeff and left_blocks / right_blocks,
# int64[n, 3] rows of (output sector, input sector, pool offset).


def _np(x):
    if hasattr(x, "detach"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


class LayoutSU2:
    """Reduced blocks (a, c) in (left sector, right sector) order."""

    def __init__(self, Lq, Ld, Rq, Rd, Q):
        self.Lq = np.asarray(Lq).reshape(-1, 2)
        self.Rq = np.asarray(Rq).reshape(-1, 2)
        self.Ld = np.asarray(Ld, dtype=np.int64)
        self.Rd = np.asarray(Rd, dtype=np.int64)
        self.N, self.tS = int(Q[0]), int(Q[1])
        self.offset = {}
        self.blocks = []
        off = 0
        for a in range(len(self.Ld)):
            for c in range(len(self.Rd)):
                if int(self.Lq[a][0]) + int(self.Rq[c][0]) != self.N:
                    continue
                if not _tri(int(self.Lq[a][1]), int(self.Rq[c][1]), self.tS):
                    continue
                self.offset[(a, c)] = off
                self.blocks.append((a, c))
                off += int(self.Ld[a] * self.Rd[c])
        self.total = off

    def block(self, vec, a, c):
        o = self.offset[(a, c)]
        return vec[o:o + int(self.Ld[a] * self.Rd[c])].reshape(int(self.Ld[a]), int(self.Rd[c]))


def layout_su2(prob):
    return LayoutSU2(prob.Lq, prob.Ld, prob.Rq, prob.Rd, prob.Q)


def term_items_su2(lay: LayoutSU2, t, tM=None):
    """(in block, out block, A, transA, B, transB, alpha) of one term, A and B
    as (pool, offset, rows, cols) of the stored reduced blocks."""
    items = []
    Lq, Rq = lay.Lq, lay.Rq
    if t.one_sided:
        stored = t.left_blocks if t.one_sided == 1 else t.right_blocks
        for (out, inp, off) in np.asarray(stored).tolist():
            for (a, c) in lay.blocks:
                side_in = a if t.one_sided == 1 else c
                if side_in != inp:
                    continue
                dst = (out, c) if t.one_sided == 1 else (a, out)
                if dst not in lay.offset:
                    continue
                d_out = int((lay.Ld if t.one_sided == 1 else lay.Rd)[out])
                d_in = int((lay.Ld if t.one_sided == 1 else lay.Rd)[inp])
                spec = ("L" if t.one_sided == 1 else "R", int(off), d_out, d_in)
                A, B = (spec, None) if t.one_sided == 1 else (None, spec)
                items.append(((a, c), dst, A, False, B, False, t.coeff))
                if t.hc:
                    items.append((dst, (a, c), A, A is not None, B, B is not None, t.coeff))
        return items
    for (a2, a, lo) in np.asarray(t.left_blocks).tolist():
        for (c2, c, ro) in np.asarray(t.right_blocks).tolist():
            if (a, c) not in lay.offset or (a2, c2) not in lay.offset:
                continue
            w = weight(int(Lq[a][1]), int(Rq[c][1]), int(Lq[a2][1]), int(Rq[c2][1]), t.two_k, lay.tS, tM)
            if w == 0.0:
                continue
            s = -1.0 if (t.odd and int(Lq[a][0]) % 2) else 1.0
            alpha = t.coeff * s * w
            A = ("L", int(lo), int(lay.Ld[a2]), int(lay.Ld[a]))
            B = ("R", int(ro), int(lay.Rd[c2]), int(lay.Rd[c]))
            items.append(((a, c), (a2, c2), A, False, B, False, alpha))
            if t.hc:
                items.append(((a2, c2), (a, c), A, True, B, True, alpha))
    return items


def _get(pools, spec, trans):
    kind, off, rows, cols = spec
    m = pools[kind][off:off + rows * cols].reshape(rows, cols)
    return m.T if trans else m


def heff_apply_su2(prob, psi=None, tM=None):
    """y = H_eff psi on the reduced blocks, float64, left-first, ascending
    terms (tM: the magnetic quantum number at which the weights are summed)."""
    lay = layout_su2(prob)
    pools = {"L": _np(prob.left_pool), "R": _np(prob.right_pool)}
    x = _np(prob.psi if psi is None else psi).astype(np.float64)
    y = np.zeros(lay.total)
    for t in prob.terms:
        for (src, dst, A, tA, B, tB, alpha) in term_items_su2(lay, t, tM):
            X = lay.block(x, *src)
            if A is not None:
                X = _get(pools, A, tA) @ X
            if B is not None:
                X = X @ _get(pools, B, tB).T
            lay.block(y, *dst)[...] += alpha * X
    return y


def heff_dense_su2(prob):
    lay = layout_su2(prob)
    H = np.zeros((lay.total, lay.total))
    for j in range(lay.total):
        e = np.zeros(lay.total)
        e[j] = 1.0
        H[:, j] = heff_apply_su2(prob, e)
    return H


def heff_diag_su2(prob):
    """Diagonal: only items whose input and output blocks coincide reach it;
    for those diag(A X B^T) at (i, j) is A_ii B_jj."""
    lay = layout_su2(prob)
    pools = {"L": _np(prob.left_pool), "R": _np(prob.right_pool)}
    d = np.zeros(lay.total)
    for t in prob.terms:
        for (src, dst, A, tA, B, tB, alpha) in term_items_su2(lay, t):
            if src != dst:
                continue
            a, c = src
            da = np.ones(int(lay.Ld[a])) if A is None else np.diag(_get(pools, A, tA))
            db = np.ones(int(lay.Rd[c])) if B is None else np.diag(_get(pools, B, tB))
            lay.block(d, a, c)[...] += alpha * np.outer(da, db)
    return d


def count_flops_su2(prob):
    """Algorithmic FLOPs: every item at its cheaper association order, one
    GEMM for one-sided items (the U(1) rule of oracle.heff.count_flops)."""
    lay = layout_su2(prob)
    total = 0
    for t in prob.terms:
        for (src, dst, A, tA, B, tB, alpha) in term_items_su2(lay, t):
            (a, c), (a2, c2) = src, dst
            dli, dri, dlo, dro = int(lay.Ld[a]), int(lay.Rd[c]), int(lay.Ld[a2]), int(lay.Rd[c2])
            if A is None:
                total += 2 * dli * dri * dro
            elif B is None:
                total += 2 * dlo * dli * dri
            else:
                total += min(2 * dlo * dli * dri + 2 * dlo * dri * dro, 2 * dli * dri * dro + 2 * dlo * dli * dro)
    return total


# ---------------------------------------------------------------------------
# The same problem in U(1) x U(1) form (for oracle.heff).


@dataclass
class _Term:
    dq: tuple
    odd: int
    hc: int
    one_sided: int
    coeff: float
    left_off: np.ndarray | None
    right_off: np.ndarray | None


@dataclass
class _Problem:
    Lq: np.ndarray
    Ld: np.ndarray
    Rq: np.ndarray
    Rd: np.ndarray
    Q: np.ndarray
    terms: list
    left_pool: np.ndarray
    right_pool: np.ndarray
    psi: np.ndarray


class _Expansion:
    """U(1) sectors (N, 2m) of one block and where each (SU(2) sector,
    m, multiplet) lands in them."""

    def __init__(self, q, d):
        q = np.asarray(q).reshape(-1, 2)
        self.sectors = []
        self.dim = []
        self.rows = {}  # (su2 sector, tm) -> (u1 sector, first row)
        index = {}
        for a in range(len(d)):
            N, tj = int(q[a][0]), int(q[a][1])
            for tm in range(-tj, tj + 1, 2):
                key = (N, tm)
                if key not in index:
                    index[key] = len(self.sectors)
                    self.sectors.append(key)
                    self.dim.append(0)
                u = index[key]
                self.rows[(a, tm)] = (u, self.dim[u])
                self.dim[u] += int(d[a])
        self.index = index


def expand_to_u1(prob, tM=None):
    """(U(1) problem, isometry function) for the states of total M (default
    M = S): the expanded operators of every term, one U(1) term per
    component q, and psi expanded through Clebsch-Gordan coefficients."""
    tS = int(prob.Q[1])
    tM = tS if tM is None else tM
    Lq = np.asarray(prob.Lq).reshape(-1, 2)
    Rq = np.asarray(prob.Rq).reshape(-1, 2)
    Ld = np.asarray(prob.Ld, dtype=np.int64)
    Rd = np.asarray(prob.Rd, dtype=np.int64)
    EL, ER = _Expansion(Lq, Ld), _Expansion(Rq, Rd)
    lay = layout_su2(prob)
    pools = {"L": _np(prob.left_pool), "R": _np(prob.right_pool)}
    Nt = int(prob.Q[0])

    # U(1) wavefunction layout (oracle.heff's own rule: one right partner per left sector)
    uLq = np.array(EL.sectors, dtype=np.int32).reshape(-1, 2)
    uRq = np.array(ER.sectors, dtype=np.int32).reshape(-1, 2)
    uLd = np.array(EL.dim, dtype=np.int64)
    uRd = np.array(ER.dim, dtype=np.int64)
    Qu = np.array([Nt, tM], dtype=np.int32)

    def expand_vec(v):
        from oracle.heff import Layout
        ul = Layout(uLq, uLd, uRq, uRd, Qu)
        out = np.zeros(ul.total)
        for (a, c) in lay.blocks:
            X = lay.block(v, a, c)
            tja, tjc = int(Lq[a][1]), int(Rq[c][1])
            for tma in range(-tja, tja + 1, 2):
                tmc = tM - tma
                if abs(tmc) > tjc or (tjc + tmc) % 2:
                    continue
                coef = cg(tja, tma, tjc, tmc, tS, tM)
                if coef == 0.0:
                    continue
                ua, ra = EL.rows[(a, tma)]
                uc, rc = ER.rows[(c, tmc)]
                assert ul.partner[ua] == uc
                blk = ul.block(out, ua)
                blk[ra:ra + int(Ld[a]), rc:rc + int(Rd[c])] += coef * X
        return out

    lpool, rpool = [], []
    lsize = rsize = 0
    terms = []
    for t in prob.terms:
        qs = [0] if t.one_sided else list(range(-t.two_k, t.two_k + 1, 2))
        for tq in qs:
            phase = 1.0 if t.one_sided else (-1.0 if ((t.two_k - tq) // 2) % 2 else 1.0)
            lo = ro = None
            if t.one_sided != 2:
                lo = np.full(len(uLq), -1, dtype=np.int64)
                blocks = {}
                for (a2, a, off) in np.asarray(t.left_blocks).tolist():
                    A = pools["L"][off:off + int(Ld[a2] * Ld[a])].reshape(int(Ld[a2]), int(Ld[a]))
                    tja, tja2 = int(Lq[a][1]), int(Lq[a2][1])
                    for tma in range(-tja, tja + 1, 2):
                        tma2 = tma + tq
                        if abs(tma2) > tja2:
                            continue
                        coef = cg(tja, tma, t.two_k, tq, tja2, tma2)
                        if coef == 0.0:
                            continue
                        ua, ra = EL.rows[(a, tma)]
                        ub, rb = EL.rows[(a2, tma2)]
                        m = blocks.setdefault(ua, (ub, np.zeros((int(uLd[ub]), int(uLd[ua])))))[1]
                        m[rb:rb + A.shape[0], ra:ra + A.shape[1]] += coef * A
                for ua, (ub, m) in blocks.items():
                    lo[ua] = lsize
                    lpool.append(m.reshape(-1))
                    lsize += m.size
            if t.one_sided != 1:
                ro = np.full(len(uRq), -1, dtype=np.int64)
                blocks = {}
                for (c2, c, off) in np.asarray(t.right_blocks).tolist():
                    B = pools["R"][off:off + int(Rd[c2] * Rd[c])].reshape(int(Rd[c2]), int(Rd[c]))
                    tjc, tjc2 = int(Rq[c][1]), int(Rq[c2][1])
                    for tmc in range(-tjc, tjc + 1, 2):
                        tmc2 = tmc - tq
                        if abs(tmc2) > tjc2:
                            continue
                        coef = cg(tjc, tmc, t.two_k, -tq, tjc2, tmc2)
                        if coef == 0.0:
                            continue
                        uc, rc = ER.rows[(c, tmc)]
                        ue, re_ = ER.rows[(c2, tmc2)]
                        m = blocks.setdefault(uc, (ue, np.zeros((int(uRd[ue]), int(uRd[uc])))))[1]
                        m[re_:re_ + B.shape[0], rc:rc + B.shape[1]] += coef * B
                for uc, (ue, m) in blocks.items():
                    ro[uc] = rsize
                    rpool.append(m.reshape(-1))
                    rsize += m.size
            terms.append(_Term(dq=(t.dn, tq), odd=t.odd, hc=t.hc, one_sided=t.one_sided,
                               coeff=t.coeff * phase, left_off=lo, right_off=ro))
    up = _Problem(uLq, uLd, uRq, uRd, Qu, terms,
                  np.concatenate(lpool) if lpool else np.zeros(1),
                  np.concatenate(rpool) if rpool else np.zeros(1),
                  expand_vec(_np(prob.psi)))
    return up, expand_vec


# ---------------------------------------------------------------------------
# Sampled entries of a whole-size problem.


@lru_cache(maxsize=None)
def _weight_cached(tja, tjc, tja2, tjc2, tk, tS):
    return weight(tja, tjc, tja2, tjc2, tk, tS)


def heff_entries_blocks_su2(prob, samples, psi=None):
    """Entries y[(a', c')][rows, cols] of y = H_eff psi for the sampled output
    blocks (samples maps (a', c') to (rows, cols)), by the definition of
    heff_apply_su2 taken item by item, with the sum of the absolute values
    of the products entering each entry (the scale of its rounding error).
    Only the items that reach a sampled block are formed, and only the
    needed rows of their operator blocks leave the pools."""
    from oracle.heff import _rows_of
    lay = layout_su2(prob)
    Lq, Rq = lay.Lq, lay.Rq
    pools = {"L": prob.left_pool, "R": prob.right_pool}
    x = _np(prob.psi if psi is None else psi).astype(np.float64)
    want = set(samples)
    groups = {}
    for t in prob.terms:
        if t.one_sided:
            stored = t.left_blocks if t.one_sided == 1 else t.right_blocks
            for (out, inp, off) in np.asarray(stored).tolist():
                for dst in want:
                    a2, c2 = dst
                    if (t.one_sided == 1 and a2 != out) or (t.one_sided == 2 and c2 != out):
                        continue
                    src = (inp, c2) if t.one_sided == 1 else (a2, inp)
                    if src not in lay.offset:
                        continue
                    d = int((lay.Ld if t.one_sided == 1 else lay.Rd)[out])
                    spec = ("L" if t.one_sided == 1 else "R", int(off), d, d)
                    A, B = (spec, None) if t.one_sided == 1 else (None, spec)
                    groups.setdefault((src, dst, t.one_sided), []).append((A, False, B, False, t.coeff))
                # hc: the transposed block carries `out`-side inputs to `inp`-side outputs
                if t.hc:
                    for dst in want:
                        a2, c2 = dst
                        if (t.one_sided == 1 and a2 != inp) or (t.one_sided == 2 and c2 != inp):
                            continue
                        src = (out, c2) if t.one_sided == 1 else (a2, out)
                        if src not in lay.offset:
                            continue
                        d = int((lay.Ld if t.one_sided == 1 else lay.Rd)[out])
                        spec = ("L" if t.one_sided == 1 else "R", int(off), d, d)
                        A, B = (spec, None) if t.one_sided == 1 else (None, spec)
                        groups.setdefault((src, dst, t.one_sided), []).append(
                            (A, A is not None, B, B is not None, t.coeff))
            continue
        # stored blocks indexed by output and by input sector
        lo_out, lo_in, ro_out, ro_in = {}, {}, {}, {}
        for (a2, a, lo) in np.asarray(t.left_blocks).tolist():
            lo_out.setdefault(a2, []).append((a, lo))
            lo_in.setdefault(a, []).append((a2, lo))
        for (c2, c, ro) in np.asarray(t.right_blocks).tolist():
            ro_out.setdefault(c2, []).append((c, ro))
            ro_in.setdefault(c, []).append((c2, ro))

        def add(a, c, a2, c2, lo, ro, back):
            # the contribution of input block (a, c) to output (a2, c2); back:
            # its transpose (input (a2, c2), output (a, c))
            w = _weight_cached(int(Lq[a][1]), int(Rq[c][1]), int(Lq[a2][1]), int(Rq[c2][1]), t.two_k, lay.tS)
            if w == 0.0:
                return
            s = -1.0 if (t.odd and int(Lq[a][0]) % 2) else 1.0
            A = ("L", int(lo), int(lay.Ld[a2]), int(lay.Ld[a]))
            B = ("R", int(ro), int(lay.Rd[c2]), int(lay.Rd[c]))
            key = ((a2, c2), (a, c), 0) if back else ((a, c), (a2, c2), 0)
            groups.setdefault(key, []).append((A, back, B, back, t.coeff * s * w))

        for (a2, c2) in want:
            for (a, lo) in lo_out.get(a2, ()):
                for (c, ro) in ro_out.get(c2, ()):
                    if (a, c) in lay.offset:
                        add(a, c, a2, c2, lo, ro, False)
            if t.hc:  # (a2, c2) as the input side of an original contribution
                for (ap, lo) in lo_in.get(a2, ()):
                    for (cp, ro) in ro_in.get(c2, ()):
                        if (ap, cp) in lay.offset:
                            add(a2, c2, ap, cp, lo, ro, True)
    out = {b: (np.zeros((len(r), len(c))), np.zeros((len(r), len(c)))) for b, (r, c) in samples.items()}
    for (src, dst, kind), items in groups.items():
        rows, cols = (list(v) for v in samples[dst])
        X = lay.block(x, *src)
        al = np.array([it[4] for it in items])
        if kind != 2:
            A_ = _rows_of(pools["L"], [it[0] for it in items], [it[1] for it in items], rows)
        if kind != 1:
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
        val, mag = out[dst]
        val += np.einsum("n,nrc->rc", al, v)
        mag += np.einsum("n,nrc->rc", np.abs(al), m)
    return out

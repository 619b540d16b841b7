// SU(2) spin-adapted form of the two-site effective Hamiltonian.
//
// The paper's DMRG is spin adapted, its bond dimensions counting multiplets
// (Introduction; Performance assessment section; P450 section).  With the
// Wigner-Eckart theorem every operator of spin rank k is stored by reduced
// blocks O[(N', j'), (N, j)] (convention <j' m'|T_q|j m> = <j m; k q|j' m'>
// times the reduced element), the wavefunction of total spin S by reduced
// blocks Psi[(a, c)] for every left sector a and right sector c whose spins
// couple to S, and the scalar term c sum_q (-1)^(k-q) T_q (x) U_{-q} acts on
// the reduced blocks as
//
//   Y[(a', c')] += c * s * W * O^L[a', a] Psi[(a, c)] O^R[c', c]^T,
//   W = (-1)^(j_a + j_c' + k + S) sqrt((2 j_a' + 1)(2 j_c' + 1))
//       { j_a'  j_c'  S }
//       { j_c   j_a   k },
//
// a Wigner 6j symbol (the recoupling of (j_a j_c) S through the two rank-k
// operators; the general coupled-tensor formula of angular-momentum theory
// with total rank 0).  s is the fermionic sign of the U(1) form.  Every item
// is therefore an ordinary sector product with the weight folded into its
// coefficient, and the grouped-GEMM programs, kernels, diagonal, adjoint and
// Davidson of the U(1) form run unchanged.  The 6j symbol is Racah's single
// sum, evaluated in long double.
#include <cmath>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "plan.h"

namespace dmrg {

namespace {

// Doubled spins throughout: tj = 2j.
bool tri(int a, int b, int c) { return std::abs(a - b) <= c && c <= a + b && ((a + b + c) & 1) == 0; }

long double fact(int two_x) {  // (two_x / 2)!
  long double r = 1.0L;
  for (int i = 2; i <= two_x / 2; ++i) r *= (long double)i;
  return r;
}

long double tri_coef(int a, int b, int c) {
  return fact(a + b - c) * fact(a - b + c) * fact(-a + b + c) / fact(a + b + c + 2);
}

// { a b c ; d e f } by Racah's formula (doubled arguments).
double six_j(int a, int b, int c, int d, int e, int f) {
  if (!tri(a, b, c) || !tri(a, e, f) || !tri(d, b, f) || !tri(d, e, c)) return 0.0;
  const long double pre = std::sqrt(tri_coef(a, b, c) * tri_coef(a, e, f) * tri_coef(d, b, f) * tri_coef(d, e, c));
  const int lo = std::max(std::max(a + b + c, a + e + f), std::max(d + b + f, d + e + c));
  const int hi = std::min(std::min(a + b + d + e, b + c + e + f), a + c + d + f);
  long double sum = 0.0L;
  for (int t = lo; t <= hi; t += 2) {
    const long double den = fact(t - a - b - c) * fact(t - a - e - f) * fact(t - d - b - f) * fact(t - d - e - c) *
                            fact(a + b + d + e - t) * fact(b + c + e + f - t) * fact(a + c + d + f - t);
    const long double term = fact(t + 2) / den;
    sum += ((t / 2) & 1) ? -term : term;
  }
  return (double)(pre * sum);
}

}  // namespace

double su2_weight(int tja, int tjc, int tja2, int tjc2, int tk, int tS) {
  const double sj = six_j(tja2, tjc2, tS, tjc, tja, tk);
  if (sj == 0.0) return 0.0;
  const int x = tja + tjc2 + tk + tS;  // even whenever the 6j symbol is non-zero
  const double ph = ((x / 2) & 1) ? -1.0 : 1.0;
  return ph * std::sqrt((double)(tja2 + 1) * (double)(tjc2 + 1)) * sj;
}

// Reduced blocks of total (N, 2S): every (a, c) with N_a + N_c = N whose
// spins couple to S, in (a, c) order.
void su2_layout(const dmrg_basis_s* L, const dmrg_basis_s* R, const int32_t Q[2],
                std::vector<BlockInfo>* blocks, int64_t* total) {
  int64_t off = 0;
  for (size_t a = 0; a < L->dim.size(); ++a)
    for (size_t c = 0; c < R->dim.size(); ++c) {
      if (L->qn[2 * a] + R->qn[2 * c] != Q[0]) continue;
      if (!tri(L->qn[2 * a + 1], R->qn[2 * c + 1], Q[1])) continue;
      if (blocks) blocks->push_back(BlockInfo{(int32_t)a, (int32_t)c, (int32_t)L->dim[a], (int32_t)R->dim[c], off});
      off += L->dim[a] * R->dim[c];
    }
  *total = off;
}

dmrg_status build_items_su2(dmrg_heff_s* h, int64_t n_terms, const dmrg_term_su2* terms) {
  const int nL = (int)h->Ld.size(), nR = (int)h->Rd.size();
  const int tS = h->Q[1];
  // block index of (a, c), and the blocks of each left sector
  std::vector<int32_t> blk((size_t)nL * nR, -1);
  std::vector<std::vector<int32_t>> of_left(nL);
  for (size_t b = 0; b < h->blocks.size(); ++b) {
    blk[(size_t)h->blocks[b].a * nR + h->blocks[b].c] = (int32_t)b;
    of_left[h->blocks[b].a].push_back((int32_t)b);
  }
  std::map<std::tuple<int, int, int, int, int>, double> wcache;
  auto W = [&](int a, int c, int a2, int c2, int tk) {
    const auto key = std::make_tuple(h->Lqn[2 * a + 1], h->Rqn[2 * c + 1], h->Lqn[2 * a2 + 1], h->Rqn[2 * c2 + 1], tk);
    auto it = wcache.find(key);
    if (it != wcache.end()) return it->second;
    const double w = su2_weight(std::get<0>(key), std::get<1>(key), std::get<2>(key), std::get<3>(key), tk, tS);
    wcache.emplace(key, w);
    return w;
  };
  struct Stored {
    int32_t out;
    int64_t off;
  };
  for (int64_t ti = 0; ti < n_terms; ++ti) {
    const dmrg_term_su2& t = terms[ti];
    const std::string where = "term " + std::to_string(ti) + ": ";
    if (t.one_sided < 0 || t.one_sided > 2 || t.reserved != 0 || (t.odd != 0 && t.odd != 1) ||
        (t.hc != 0 && t.hc != 1) || t.two_k < 0 || !std::isfinite(t.coeff) || t.n_left < 0 || t.n_right < 0)
      return fail(DMRG_EINVAL, where + "bad flags, rank or coefficient");
    if (t.one_sided && (t.two_k != 0 || t.dn != 0 || t.odd))
      return fail(DMRG_EQN, where + "a one-sided term must be a scalar (two_k = 0) with dn = 0 and even parity");
    if (t.odd != (std::abs(t.dn) % 2))
      return fail(DMRG_EQN, where + "parity flag does not match the particle-number shift");
    const bool hasL = t.one_sided != 2, hasR = t.one_sided != 1;
    if ((hasL && t.n_left > 0 && !t.left_blocks) || (hasR && t.n_right > 0 && !t.right_blocks))
      return fail(DMRG_EINVAL, where + "missing block table");
    // stored blocks by input sector, checked against the selection rules and the pools
    std::vector<std::vector<Stored>> lin(nL), rin(nR);
    for (int side = 0; side < 2; ++side) {
      if ((side == 0 && !hasL) || (side == 1 && !hasR)) continue;
      const int64_t n = side == 0 ? t.n_left : t.n_right;
      const int64_t* tab = side == 0 ? t.left_blocks : t.right_blocks;
      const int ns = side == 0 ? nL : nR;
      const std::vector<int32_t>& qn = side == 0 ? h->Lqn : h->Rqn;
      const std::vector<int64_t>& dim = side == 0 ? h->Ld : h->Rd;
      const int dn = side == 0 ? t.dn : -t.dn;
      for (int64_t i = 0; i < n; ++i) {
        const int64_t out = tab[3 * i], in = tab[3 * i + 1], off = tab[3 * i + 2];
        if (out < 0 || out >= ns || in < 0 || in >= ns || off < 0)
          return fail(DMRG_EINVAL, where + "block " + std::to_string(i) + " names a sector outside the basis");
        if (qn[2 * out] - qn[2 * in] != dn || !tri(qn[2 * in + 1], t.two_k, qn[2 * out + 1]))
          return fail(DMRG_EQN, where + "block " + std::to_string(i) + " breaks the selection rules");
        if (off + dim[out] * dim[in] > (side == 0 ? h->llen : h->rlen))
          return fail(DMRG_EQN, where + "block " + std::to_string(i) + " outside its pool");
        (side == 0 ? lin : rin)[in].push_back(Stored{(int32_t)out, off});
      }
    }
    for (size_t bi = 0; bi < h->blocks.size(); ++bi) {
      const BlockInfo& B = h->blocks[bi];
      Item it{};
      it.term = (int32_t)ti;
      it.in = (int32_t)bi;
      if (t.one_sided == 1) {
        for (const Stored& s : lin[B.a]) {  // scalar, dn = 0: s.out == B.a
          it.out = blk[(size_t)s.out * nR + B.c];
          if (it.out < 0) continue;
          it.aoff = s.off;
          it.arows = (int32_t)h->Ld[s.out];
          it.acols = B.dl;
          it.boff = -1;
          it.kind = 1;
          it.alpha = t.coeff;
          it.at = 0;
          h->items.push_back(it);
          if (t.hc) {
            Item p = it;
            std::swap(p.in, p.out);
            p.at = 1;
            h->items.push_back(p);
          }
        }
        continue;
      }
      if (t.one_sided == 2) {
        for (const Stored& s : rin[B.c]) {
          it.out = blk[(size_t)B.a * nR + s.out];
          if (it.out < 0) continue;
          it.aoff = -1;
          it.boff = s.off;
          it.brows = (int32_t)h->Rd[s.out];
          it.bcols = B.dr;
          it.kind = 2;
          it.alpha = t.coeff;
          it.bt = 0;
          h->items.push_back(it);
          if (t.hc) {
            Item p = it;
            std::swap(p.in, p.out);
            p.bt = 1;
            h->items.push_back(p);
          }
        }
        continue;
      }
      const double s_in = (t.odd && (h->Lqn[2 * B.a] & 1)) ? -1.0 : 1.0;
      for (const Stored& l : lin[B.a])
        for (const Stored& r : rin[B.c]) {
          const int32_t ob = blk[(size_t)l.out * nR + r.out];
          if (ob < 0) continue;
          const double w = W(B.a, B.c, l.out, r.out, t.two_k);
          if (w == 0.0) continue;
          Item x{};
          x.term = (int32_t)ti;
          x.in = (int32_t)bi;
          x.out = ob;
          x.aoff = l.off;
          x.arows = (int32_t)h->Ld[l.out];
          x.acols = B.dl;
          x.boff = r.off;
          x.brows = (int32_t)h->Rd[r.out];
          x.bcols = B.dr;
          x.kind = 0;
          x.alpha = t.coeff * s_in * w;
          h->items.push_back(x);
          if (t.hc) {
            Item p = x;
            std::swap(p.in, p.out);
            p.at = p.bt = 1;
            h->items.push_back(p);
          }
        }
    }
  }
  return DMRG_OK;
}

}  // namespace dmrg

extern "C" {

double dmrg_su2_weight(int32_t two_ja, int32_t two_jc, int32_t two_ja2, int32_t two_jc2, int32_t two_k,
                       int32_t two_s) {
  if (two_ja < 0 || two_jc < 0 || two_ja2 < 0 || two_jc2 < 0 || two_k < 0 || two_s < 0) return 0.0;
  return dmrg::su2_weight(two_ja, two_jc, two_ja2, two_jc2, two_k, two_s);
}

dmrg_status dmrg_wfn_layout_su2(dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2], int64_t* n_blocks,
                                int32_t* block_left, int32_t* block_right, int64_t* block_offset,
                                int64_t* total) {
  if (!L || !R || !Q || !n_blocks || !total) return dmrg::fail(DMRG_EINVAL, "wfn_layout_su2: bad arguments");
  if (Q[1] < 0) return dmrg::fail(DMRG_EINVAL, "wfn_layout_su2: 2S must be >= 0");
  std::vector<dmrg::BlockInfo> b;
  dmrg::su2_layout(L, R, Q, &b, total);
  *n_blocks = (int64_t)b.size();
  for (size_t i = 0; i < b.size(); ++i) {
    if (block_left) block_left[i] = b[i].a;
    if (block_right) block_right[i] = b[i].c;
    if (block_offset) block_offset[i] = b[i].off;
  }
  return DMRG_OK;
}

}  // extern "C"

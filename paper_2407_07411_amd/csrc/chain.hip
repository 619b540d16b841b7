// Operator blocks of the ab initio Hamiltonian and the two-site sweep.
//
// The paper's DMRG sweeps over the orbital chain, updating two MPS tensors at
// a time (Numerical procedure section); each update needs the operators of
// the enlarged left block (left block + site l) and of the enlarged right
// block (site l+1 + right block) in their renormalised bases.  This file keeps
// those operators the textbook DMRG way (normal and complementary operators,
// grown one site at a time and renormalised with the SVD factors):
//
//   left block:  H, every product of one or two creation/annihilation
//                operators on its orbitals, and for every operator x outside
//                it the complementary sum C3[x] of its three-operator parts;
//   right block: H, the same one- and two-operator products, and for every
//                operator x outside it the complementary sum C13[x] of its one-
//                and three-operator parts.
//
// Growing a block by a site multiplies stored block operators with 4x4 site
// operators (Jordan-Wigner sign from the input state of the part that is
// passed); every monomial of H is sorted by where its factors live.  The
// two-site H_eff pairs are then
//   H_L (x) 1,  1 (x) H_R,  x (x) C13_R[x] for one-operator x on the left,
//   z (x) E_z for two-operator z on the left (E_z a sum of right products),
//   C3_L[y] (x) y for one-operator y on the right,
// handed to the grouped-GEMM plan; Davidson, SVD truncation and the
// renormalisation O <- U^T O U close the step.  The growth (block operators
// times 4x4 site operators, placed into the enlarged blocks) runs on the
// host; the renormalisation of every operator, H_eff, Davidson and the SVD
// run in the library's kernels when the chain has a context (the
// renormalisation as two grouped-GEMM phases, T = O U_in and U_out^T T, over
// all operators of the block at once).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <random>
#include <vector>

#include "plan.h"

namespace dmrg {
namespace {

// A creation/annihilation factor: bit 7 dagger, bits 1..6 orbital, bit 0 spin.
using Fac = uint8_t;
inline Fac mkfac(int dag, int orb, int spin) { return (Fac)((dag << 7) | (orb << 1) | spin); }
inline int fdag(Fac f) { return f >> 7; }
inline int forb(Fac f) { return (f >> 1) & 63; }
inline int fspin(Fac f) { return f & 1; }
using Key = std::vector<Fac>;

struct QN {
  int n, s;  // N, 2Sz
  bool operator<(const QN& o) const { return n != o.n ? n < o.n : s < o.s; }
  bool operator==(const QN& o) const { return n == o.n && s == o.s; }
};

QN shift_of(const Key& k) {
  QN d{0, 0};
  for (Fac f : k) {
    const int sg = fdag(f) ? 1 : -1;
    d.n += sg;
    d.s += sg * (fspin(f) == 0 ? 1 : -1);
  }
  return d;
}

// Sector-blocked operator with a fixed shift: blk[in] is d_out x d_in.
struct Op {
  QN dq{0, 0};
  std::vector<std::vector<double>> blk;
};

struct Basis {
  std::vector<QN> qn;
  std::vector<int> dim;
  int find(QN q) const {
    for (size_t i = 0; i < qn.size(); ++i)
      if (qn[i] == q) return (int)i;
    return -1;
  }
  int out_of(int in, QN dq) const { return find(QN{qn[in].n + dq.n, qn[in].s + dq.s}); }
};

struct Block {
  Basis b;
  std::vector<int> orbs;
  Op H;
  std::map<Key, Op> ops;    // one- and two-factor products
  std::map<Fac, Op> comp;   // complementary sums keyed by an outside factor
};

// Site states |0>, |up>, |dn>, |updn> = n_up + 2 n_dn; up before dn.
const QN SITE_QN[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};

// 4x4 matrix of a product of site factors (all on one orbital), row-major.
std::vector<double> site_matrix(const Key& k) {
  std::vector<double> M(16, 0.0);
  for (int x = 0; x < 4; ++x) M[x * 4 + x] = 1.0;
  for (int fi = (int)k.size() - 1; fi >= 0; --fi) {  // rightmost factor acts first
    const Fac f = k[fi];
    const int bit = 1 << fspin(f);
    std::vector<double> F(16, 0.0);
    for (int x = 0; x < 4; ++x) {
      const bool occ = x & bit;
      if (fdag(f) == occ) continue;  // a+ on occupied or a on empty
      const int y = x ^ bit;
      const double sg = (fspin(f) == 1 && (x & 1)) ? -1.0 : 1.0;  // pass the up mode
      F[y * 4 + x] = sg;
    }
    std::vector<double> R(16, 0.0);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int l = 0; l < 4; ++l) R[i * 4 + j] += F[i * 4 + l] * M[l * 4 + j];
    M = R;
  }
  return M;
}

// Reorder factors so that those with pred() come first (relative order kept);
// returns the sign of the permutation.
template <class P>
double split(const Key& k, P&& pred, Key& first, Key& second) {
  first.clear();
  second.clear();
  int inv = 0, seen_second = 0;
  for (Fac f : k) {
    if (pred(f)) {
      first.push_back(f);
      inv += seen_second;
    } else {
      second.push_back(f);
      ++seen_second;
    }
  }
  return (inv & 1) ? -1.0 : 1.0;
}

// Enlarged basis of (block x site) or (site x block): sector list plus, per
// enlarged sector, the offset of every (block sector, site state) piece.
struct Enlarged {
  Basis b;
  std::vector<std::vector<int>> off;  // off[e][bsec*4 + s] or -1
  std::vector<int> sec;               // enlarged sector of piece bsec*4 + s
};

Enlarged enlarge(const Basis& B, bool site_first) {
  Enlarged E;
  std::map<QN, int> idx;
  for (size_t bs = 0; bs < B.qn.size(); ++bs)
    for (int s = 0; s < 4; ++s) idx[QN{B.qn[bs].n + SITE_QN[s].n, B.qn[bs].s + SITE_QN[s].s}] = 0;
  for (auto& kv : idx) {
    kv.second = (int)E.b.qn.size();
    E.b.qn.push_back(kv.first);
  }
  E.b.dim.assign(E.b.qn.size(), 0);
  E.off.assign(E.b.qn.size(), std::vector<int>(B.qn.size() * 4, -1));
  E.sec.assign(B.qn.size() * 4, -1);
  auto place = [&](int bs, int s) {
    const int e = idx[QN{B.qn[bs].n + SITE_QN[s].n, B.qn[bs].s + SITE_QN[s].s}];
    E.sec[bs * 4 + s] = e;
    E.off[e][bs * 4 + s] = E.b.dim[e];
    E.b.dim[e] += B.dim[bs];
  };
  if (!site_first) {
    for (size_t bs = 0; bs < B.qn.size(); ++bs)
      for (int s = 0; s < 4; ++s) place((int)bs, s);
  } else {
    for (int s = 0; s < 4; ++s)
      for (size_t bs = 0; bs < B.qn.size(); ++bs) place((int)bs, s);
  }
  return E;
}

Op zero_op(const Basis& b, QN dq) {
  Op o;
  o.dq = dq;
  o.blk.resize(b.qn.size());
  return o;
}

// E += c * (B-part (x) S-part) on the enlarged basis.  bop == nullptr means
// the identity on the block; the sign (-1)^{N(passed input)} follows the
// Jordan-Wigner order (left growth: the site part passes the block state;
// right growth: the block part passes the site state).
void add_kron(Op& E, const Enlarged& en, const Basis& B, bool site_first, double c, const Op* bop,
              const std::vector<double>& S, int s_parity, int b_parity) {
  for (size_t bs = 0; bs < B.qn.size(); ++bs) {
    int bo = (int)bs;
    const std::vector<double>* blk = nullptr;
    if (bop) {
      if (bop->blk[bs].empty()) continue;
      bo = B.out_of((int)bs, bop->dq);
      if (bo < 0) continue;
      blk = &bop->blk[bs];
    }
    const int din = B.dim[bs], dout = B.dim[bo];
    for (int si = 0; si < 4; ++si)
      for (int so = 0; so < 4; ++so) {
        const double sv = S[so * 4 + si];
        if (sv == 0.0) continue;
        double sg = 1.0;
        if (!site_first && s_parity && (B.qn[bs].n & 1)) sg = -1.0;
        if (site_first && b_parity && (SITE_QN[si].n & 1)) sg = -1.0;
        const int e_in = en.sec[bs * 4 + si], e_out = en.sec[bo * 4 + so];
        auto& tgt = E.blk[e_in];
        const int Din = en.b.dim[e_in], Dout = en.b.dim[e_out];
        if (tgt.empty()) tgt.assign((size_t)Dout * Din, 0.0);
        const int r0 = en.off[e_out][bo * 4 + so], c0 = en.off[e_in][bs * 4 + si];
        const double f = c * sg * sv;
        for (int i = 0; i < dout; ++i)
          for (int j = 0; j < din; ++j) {
            const double v = blk ? (*blk)[(size_t)i * din + j] : (i == j ? 1.0 : 0.0);
            if (v != 0.0) tgt[(size_t)(r0 + i) * Din + (c0 + j)] += f * v;
          }
      }
  }
}

// O' = Uout^T O Uin for every block; U[sec] is d x k row-major (k = kept[sec]).
Op renorm(const Op& O, const Basis& from, const Basis& to, const std::vector<int>& map_to,
          const std::vector<std::vector<double>>& U) {
  Op R = zero_op(to, O.dq);
  for (size_t in = 0; in < from.qn.size(); ++in) {
    if (O.blk[in].empty() || map_to[in] < 0) continue;
    const int out = from.out_of((int)in, O.dq);
    if (out < 0 || map_to[out] < 0) continue;
    const int din = from.dim[in], dout = from.dim[out];
    const int kin = to.dim[map_to[in]], kout = to.dim[map_to[out]];
    std::vector<double> tmp((size_t)dout * kin, 0.0);  // O Uin
    for (int i = 0; i < dout; ++i)
      for (int l = 0; l < din; ++l) {
        const double v = O.blk[in][(size_t)i * din + l];
        if (v == 0.0) continue;
        for (int j = 0; j < kin; ++j) tmp[(size_t)i * kin + j] += v * U[in][(size_t)l * kin + j];
      }
    std::vector<double> r((size_t)kout * kin, 0.0);
    for (int i = 0; i < dout; ++i)
      for (int a = 0; a < kout; ++a) {
        const double u = U[out][(size_t)i * kout + a];
        if (u == 0.0) continue;
        for (int j = 0; j < kin; ++j) r[(size_t)a * kin + j] += u * tmp[(size_t)i * kin + j];
      }
    R.blk[map_to[in]] = std::move(r);
  }
  return R;
}

struct Monomial {
  double c;
  Key f;
};

}  // namespace
}  // namespace dmrg

using namespace dmrg;

struct dmrg_chain_s {
  dmrg_ctx_t ctx = nullptr;
  int L = 0, n_elec = 0, two_sz = 0;
  int64_t D = 0;
  std::vector<Monomial> H;            // every monomial of the Hamiltonian
  std::vector<Block> left;            // left[l]: orbitals [0, l)
  std::vector<Block> right;           // right[j]: orbitals [j, L)
  std::mt19937_64 rng;
};

namespace {

bool compatible(const dmrg_chain_s* c, QN q, int n_orb_other) {
  // alpha / beta counts of this part and of the complement
  if ((q.n + q.s) & 1) return false;
  const int na = (q.n + q.s) / 2, nb = (q.n - q.s) / 2;
  const int Na = (c->n_elec + c->two_sz) / 2, Nb = (c->n_elec - c->two_sz) / 2;
  const int ra = Na - na, rb = Nb - nb;
  return na >= 0 && nb >= 0 && ra >= 0 && rb >= 0 && ra <= n_orb_other && rb <= n_orb_other;
}

// Grow block B by orbital o (left growth: site after the block; right
// growth: site before it).  Returns the enlarged block with every stored
// operator rebuilt; ok = false if a needed block product is missing.
Block grow(const dmrg_chain_s* c, const Block& B, int o, bool site_first, bool* ok) {
  Enlarged en = enlarge(B.b, site_first);
  Block E;
  E.b = en.b;
  E.orbs = B.orbs;
  E.orbs.push_back(o);
  std::sort(E.orbs.begin(), E.orbs.end());
  const bool left_block = !site_first;
  auto in_B = [&](Fac f) { return std::binary_search(B.orbs.begin(), B.orbs.end(), forb(f)); };
  auto in_E = [&](Fac f) { return std::binary_search(E.orbs.begin(), E.orbs.end(), forb(f)); };
  auto on_site = [&](Fac f) { return forb(f) == o; };
  *ok = true;

  // tgt += cf * (block part)(site part) in the growth order
  auto add = [&](Op& tgt, double cf, const Key& bk, const Key& sk) {
    const Op* bo = nullptr;
    if (bk.size() == 2 && bk[0] == bk[1]) return;  // a repeated fermion factor: zero
    if (!bk.empty()) {
      auto it = B.ops.find(bk);
      if (it == B.ops.end()) {
        *ok = false;
        return;
      }
      bo = &it->second;
    }
    add_kron(tgt, en, B.b, site_first, cf, bo, site_matrix(sk), (int)(sk.size() & 1),
             (int)(bk.size() & 1));
  };
  // (block)(site) for left growth, (site)(block) for right growth
  auto parts = [&](const Key& k, Key& bk, Key& sk) -> double {
    if (left_block) return split(k, in_B, bk, sk);
    return split(k, on_site, sk, bk);
  };

  // one- and two-factor products on E
  std::vector<Fac> facs;
  for (int orb : E.orbs)
    for (int sp = 0; sp < 2; ++sp)
      for (int dg = 0; dg < 2; ++dg) facs.push_back(mkfac(dg, orb, sp));
  auto build_key = [&](const Key& k) {
    Op op = zero_op(E.b, shift_of(k));
    Key bk, sk;
    const double sg = parts(k, bk, sk);
    add(op, sg, bk, sk);
    E.ops[k] = std::move(op);
  };
  for (Fac f : facs) build_key(Key{f});
  for (Fac f : facs)
    for (Fac g : facs)
      if (f != g) build_key(Key{f, g});

  // complementary operators of E for outside factors x
  auto comp_op = [&](Fac x) -> Op& {
    auto it = E.comp.find(x);
    if (it != E.comp.end()) return it->second;
    const QN dq = shift_of(Key{x});
    return E.comp[x] = zero_op(E.b, QN{-dq.n, -dq.s});
  };
  // parts entirely inside B come from B's own complement
  for (auto& kv : B.comp) {
    if (in_E(kv.first)) continue;
    add_kron(comp_op(kv.first), en, B.b, site_first, 1.0, &kv.second, site_matrix(Key{}), 0, 1);
  }

  // H_E = H_B (x) 1 + terms inside E touching the site
  E.H = zero_op(E.b, QN{0, 0});
  add_kron(E.H, en, B.b, site_first, 1.0, &B.H, site_matrix(Key{}), 0, 0);
  for (const Monomial& m : c->H) {
    int nE = 0, nS = 0, nOut = 0;
    Fac x = 0;
    for (Fac f : m.f) {
      if (in_E(f)) {
        ++nE;
        if (on_site(f)) ++nS;
      } else {
        ++nOut;
        x = f;
      }
    }
    if (nS == 0) continue;  // without the site: already in B's operators
    Key bk, sk;
    if (nOut == 0) {
      if (nS == 1 && nE - nS == 3 && left_block) continue;  // from C3_B[site factor] below
      if (nS == 1 && nE - nS >= 1 && !left_block) continue;  // from C13_B[site factor] below
      const double sg = parts(m.f, bk, sk);
      add(E.H, m.c * sg, bk, sk);
    } else if (nOut == 1) {
      Key in, out;
      double sg;
      if (left_block) {
        if (nE != 3) continue;  // one-factor parts pair with the right complement
        sg = split(m.f, in_E, in, out);                                 // (inside)(x)
      } else {
        sg = split(m.f, [&](Fac f) { return !in_E(f); }, out, in);      // (x)(inside)
      }
      sg *= parts(in, bk, sk);
      add(comp_op(x), m.c * sg, bk, sk);
    }
  }
  // H_E terms with one site factor and the other factors in B, through B's
  // complement keyed by that site factor: (C3_B[x])(x) on the left,
  // (x)(C13_B[x]) on the right (one or three block factors)
  for (auto& kv : B.comp) {
    const Fac x = kv.first;
    if (!on_site(x)) continue;
    add_kron(E.H, en, B.b, site_first, 1.0, &kv.second, site_matrix(Key{x}), 1, 1);
  }
  return E;
}

}  // namespace

namespace {

std::vector<Monomial> hamiltonian(int L, const double* h, const double* V) {
  std::vector<Monomial> out;
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q) {
      const double v = h[p * L + q];
      if (v != 0.0)
        for (int sg = 0; sg < 2; ++sg) out.push_back(Monomial{v, Key{mkfac(1, p, sg), mkfac(0, q, sg)}});
    }
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q)
      for (int r = 0; r < L; ++r)
        for (int t = 0; t < L; ++t) {
          const double v = V[((p * L + q) * L + r) * L + t];
          if (v == 0.0) continue;
          for (int s1 = 0; s1 < 2; ++s1)
            for (int s2 = 0; s2 < 2; ++s2)
              out.push_back(Monomial{0.5 * v, Key{mkfac(1, p, s1), mkfac(1, r, s2), mkfac(0, t, s2),
                                                  mkfac(0, q, s1)}});
        }
  return out;
}

// Keep only sectors whose complement (n_other orbitals) can host the rest of
// the charge; returns the old->new sector map (-1 dropped).
std::vector<int> prune(const dmrg_chain_s* c, const Basis& b, int n_other, Basis& kept) {
  std::vector<int> map(b.qn.size(), -1);
  for (size_t i = 0; i < b.qn.size(); ++i)
    if (compatible(c, b.qn[i], n_other)) {
      map[i] = (int)kept.qn.size();
      kept.qn.push_back(b.qn[i]);
      kept.dim.push_back(b.dim[i]);
    }
  return map;
}

// Restrict every operator of a block to kept sectors with isometries U[sec]
// (d x k row-major; identity when U is empty and k == d).
Block renorm_block(const Block& E, const Basis& to, const std::vector<int>& map_to,
                   const std::vector<std::vector<double>>& U) {
  Block B;
  B.b = to;
  B.orbs = E.orbs;
  B.H = renorm(E.H, E.b, to, map_to, U);
  for (auto& kv : E.ops) B.ops[kv.first] = renorm(kv.second, E.b, to, map_to, U);
  for (auto& kv : E.comp) B.comp[kv.first] = renorm(kv.second, E.b, to, map_to, U);
  return B;
}

// The same renormalisation on the device: for every (operator, input sector)
// pair the two products T = O U_in and O' = U_out^T T run as the two phases
// of one grouped-GEMM program (the matvec's kernels), with the operator
// blocks, the isometries and the results in device buffers.
dmrg_status renorm_block_dev(dmrg_ctx_t ctx, const Block& E, const Basis& to, const std::vector<int>& map_to,
                             const std::vector<std::vector<double>>& U, Block* out) {
  std::vector<const Op*> ops{&E.H};
  for (auto& kv : E.ops) ops.push_back(&kv.second);
  for (auto& kv : E.comp) ops.push_back(&kv.second);
  std::vector<double> opool, upool;
  std::vector<int64_t> uoff(E.b.qn.size(), -1);
  for (size_t sec = 0; sec < E.b.qn.size(); ++sec)
    if (map_to[sec] >= 0) {
      uoff[sec] = (int64_t)upool.size();
      upool.insert(upool.end(), U[sec].begin(), U[sec].end());
    }
  struct Job {
    int op, in, out;
    int64_t ooff, toff, roff;
  };
  std::vector<Job> jobs;
  int64_t work = 0, res = 0;
  for (size_t o = 0; o < ops.size(); ++o) {
    const Op& O = *ops[o];
    for (size_t in = 0; in < E.b.qn.size(); ++in) {
      if (O.blk[in].empty() || map_to[in] < 0) continue;
      const int outs = E.b.out_of((int)in, O.dq);
      if (outs < 0 || map_to[outs] < 0) continue;
      const int dout = E.b.dim[outs], kin = to.dim[map_to[in]], kout = to.dim[map_to[outs]];
      jobs.push_back(Job{(int)o, (int)in, outs, (int64_t)opool.size(), work, res});
      opool.insert(opool.end(), O.blk[in].begin(), O.blk[in].end());
      work += (int64_t)dout * kin;
      res += (int64_t)kout * kin;
    }
  }
  Block R;
  R.b = to;
  R.orbs = E.orbs;
  R.H = zero_op(to, E.H.dq);
  for (auto& kv : E.ops) R.ops[kv.first] = zero_op(to, kv.second.dq);
  for (auto& kv : E.comp) R.comp[kv.first] = zero_op(to, kv.second.dq);
  std::vector<Op*> outs{&R.H};
  for (auto& kv : R.ops) outs.push_back(&kv.second);
  for (auto& kv : R.comp) outs.push_back(&kv.second);
  if (jobs.empty()) {
    *out = std::move(R);
    return DMRG_OK;
  }
  ProgramBuilder pb;
  for (const Job& j : jobs) {  // T = O U_in (dout x kin), K = din
    const int din = E.b.dim[j.in], dout = E.b.dim[j.out], kin = to.dim[map_to[j.in]];
    const int32_t pr = pb.add_prob(BUF_WORK, j.toff, dout, kin, kin, false);
    pb.add_seg(pr, make_seg(BUF_LPOOL, j.ooff, din, false, BUF_RPOOL, uoff[j.in], kin, false, din, 1.0));
  }
  pb.phase_id = 0;
  pb.close_phase();
  for (const Job& j : jobs) {  // O' = U_out^T T (kout x kin), K = dout
    const int dout = E.b.dim[j.out], kin = to.dim[map_to[j.in]], kout = to.dim[map_to[j.out]];
    const int32_t pr = pb.add_prob(BUF_Y, j.roff, kout, kin, kin, false);
    pb.add_seg(pr, make_seg(BUF_RPOOL, uoff[j.out], kout, true, BUF_WORK, j.toff, kin, false, dout, 1.0));
  }
  pb.phase_id = 1;
  pb.close_phase();
  Program& P = pb.prog;
  int64_t len[BUF_COUNT] = {0, res, (int64_t)opool.size(), (int64_t)upool.size(), work, 0, 0, 0, P.part_elems};
  dmrg_status st = P.validate(len);
  if (st != DMRG_OK) return st;
  double *dO = nullptr, *dU = nullptr, *dT = nullptr, *dR = nullptr, *dP = nullptr;
  auto cleanup = [&]() {
    P.release();
    for (double* q : {dO, dU, dT, dR, dP})
      if (q) (void)hipFree(q);
  };
  if (hipMalloc(&dO, opool.size() * 8) != hipSuccess || hipMalloc(&dU, upool.size() * 8) != hipSuccess ||
      hipMalloc(&dT, work * 8) != hipSuccess || hipMalloc(&dR, res * 8) != hipSuccess ||
      hipMalloc(&dP, std::max<int64_t>(P.part_elems, 1) * 8) != hipSuccess) {
    cleanup();
    return fail(DMRG_ENOMEM, "chain: renormalisation buffers");
  }
  hipStream_t s = ctx->stream;
  if ((st = P.upload()) == DMRG_OK) {
    Bases b{};
    b.p[BUF_Y] = dR;
    b.p[BUF_LPOOL] = dO;
    b.p[BUF_RPOOL] = dU;
    b.p[BUF_WORK] = dT;
    b.p[BUF_PART] = dP;
    for (int k = 0; k < BUF_COUNT; ++k) b.len[k] = len[k];
    std::vector<double> host(res);
    if (hipMemcpyAsync(dO, opool.data(), opool.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dU, upool.data(), upool.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      st = fail(DMRG_EHIP, "chain: renormalisation copy");
    if (st == DMRG_OK) st = P.run(b, s, DMRG_FP64);
    if (st == DMRG_OK && (hipMemcpyAsync(host.data(), dR, res * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                          hipStreamSynchronize(s) != hipSuccess))
      st = fail(DMRG_EHIP, "chain: renormalisation copy");
    if (st == DMRG_OK) {
      for (const Job& j : jobs) {
        const int kin = to.dim[map_to[j.in]], kout = to.dim[map_to[j.out]];
        outs[j.op]->blk[map_to[j.in]].assign(host.begin() + j.roff, host.begin() + j.roff + (int64_t)kout * kin);
      }
      *out = std::move(R);
    }
  }
  cleanup();
  return st;
}

// Host (DMRG_CHAIN_HOST_RENORM=1) or device renormalisation.
dmrg_status renorm_any(dmrg_ctx_t ctx, const Block& E, const Basis& to, const std::vector<int>& map_to,
                       const std::vector<std::vector<double>>& U, Block* out) {
  const char* e = std::getenv("DMRG_CHAIN_HOST_RENORM");
  if (!ctx || (e && std::atoi(e) != 0)) {
    *out = renorm_block(E, to, map_to, U);
    return DMRG_OK;
  }
  return renorm_block_dev(ctx, E, to, map_to, U, out);
}

std::vector<double> identity(int d) {
  std::vector<double> I((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) I[(size_t)i * d + i] = 1.0;
  return I;
}

// Orthonormal columns of a random d x k matrix (modified Gram-Schmidt, twice).
std::vector<double> random_isometry(std::mt19937_64& rng, int d, int k) {
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> Q((size_t)d * k);
  for (auto& x : Q) x = nd(rng);
  for (int j = 0; j < k; ++j)
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        double dot = 0.0;
        for (int r = 0; r < d; ++r) dot += Q[(size_t)r * k + i] * Q[(size_t)r * k + j];
        for (int r = 0; r < d; ++r) Q[(size_t)r * k + j] -= dot * Q[(size_t)r * k + i];
      }
      double nrm = 0.0;
      for (int r = 0; r < d; ++r) nrm += Q[(size_t)r * k + j] * Q[(size_t)r * k + j];
      nrm = std::sqrt(nrm);
      for (int r = 0; r < d; ++r) Q[(size_t)r * k + j] /= nrm;
    }
  return Q;
}

Block empty_block() {
  Block B;
  B.b.qn.push_back(QN{0, 0});
  B.b.dim.push_back(1);
  B.H.dq = QN{0, 0};
  B.H.blk.assign(1, std::vector<double>(1, 0.0));
  return B;
}

// Host pools and terms of the two-site problem at sites (l, l+1).
struct TwoSite {
  Basis Lb, Rb;
  std::vector<double> lpool, rpool;
  std::vector<dmrg_term> terms;
  std::vector<std::vector<int64_t>> loff, roff;
};

// Append an operator to a pool; offsets per input sector (-1 absent).
std::vector<int64_t> put_op(std::vector<double>& pool, const Op& o) {
  std::vector<int64_t> off(o.blk.size(), -1);
  for (size_t i = 0; i < o.blk.size(); ++i) {
    if (o.blk[i].empty()) continue;
    bool nz = false;
    for (double v : o.blk[i])
      if (v != 0.0) {
        nz = true;
        break;
      }
    if (!nz) continue;
    off[i] = (int64_t)pool.size();
    pool.insert(pool.end(), o.blk[i].begin(), o.blk[i].end());
  }
  return off;
}

bool op_is_zero(const Op& o) {
  for (auto& b : o.blk)
    for (double v : b)
      if (v != 0.0) return false;
  return true;
}

void assemble(const dmrg_chain_s* c, const Block& Le, const Block& Re, TwoSite& ts) {
  ts.Lb = Le.b;
  ts.Rb = Re.b;
  auto in_L = [&](Fac f) { return std::binary_search(Le.orbs.begin(), Le.orbs.end(), forb(f)); };
  auto add_term = [&](const Op* lo, const Op* ro, QN dq, int odd, int one_sided) {
    dmrg_term t{};
    t.dq[0] = dq.n;
    t.dq[1] = dq.s;
    t.odd = odd;
    t.hc = 0;
    t.one_sided = one_sided;
    t.coeff = 1.0;
    ts.loff.push_back(lo ? put_op(ts.lpool, *lo) : std::vector<int64_t>());
    ts.roff.push_back(ro ? put_op(ts.rpool, *ro) : std::vector<int64_t>());
    ts.terms.push_back(t);
  };
  add_term(&Le.H, nullptr, QN{0, 0}, 0, 1);
  add_term(nullptr, &Re.H, QN{0, 0}, 0, 2);
  // x (x) C13_R[x] for one-factor x on the left
  for (auto& kv : Le.ops) {
    if (kv.first.size() != 1) continue;
    auto it = Re.comp.find(kv.first[0]);
    if (it == Re.comp.end() || op_is_zero(it->second)) continue;
    add_term(&kv.second, &it->second, kv.second.dq, 1, 0);
  }
  // z (x) E_z: two factors on each side
  std::map<Key, std::map<Key, double>> zc;
  for (const Monomial& m : c->H) {
    int nl = 0;
    for (Fac f : m.f) nl += in_L(f) ? 1 : 0;
    if (m.f.size() != 4 || nl != 2) continue;
    Key lk, rk;
    const double sg = split(m.f, in_L, lk, rk);
    zc[lk][rk] += m.c * sg;
  }
  for (auto& kv : zc) {
    auto lit = Le.ops.find(kv.first);
    if (lit == Le.ops.end()) continue;
    Op E = zero_op(Re.b, QN{-lit->second.dq.n, -lit->second.dq.s});
    for (auto& rv : kv.second) {
      auto rit = Re.ops.find(rv.first);
      if (rit == Re.ops.end() || rv.second == 0.0) continue;
      const Op& ro = rit->second;
      for (size_t i = 0; i < ro.blk.size(); ++i) {
        if (ro.blk[i].empty()) continue;
        if (E.blk[i].empty()) E.blk[i].assign(ro.blk[i].size(), 0.0);
        for (size_t e = 0; e < ro.blk[i].size(); ++e) E.blk[i][e] += rv.second * ro.blk[i][e];
      }
    }
    if (op_is_zero(E)) continue;
    add_term(&lit->second, &E, lit->second.dq, 0, 0);
  }
  // C3_L[y] (x) y for one-factor y on the right
  for (auto& kv : Re.ops) {
    if (kv.first.size() != 1) continue;
    auto it = Le.comp.find(kv.first[0]);
    if (it == Le.comp.end() || op_is_zero(it->second)) continue;
    add_term(&it->second, &kv.second, it->second.dq, 1, 0);
  }
  for (size_t i = 0; i < ts.terms.size(); ++i) {
    ts.terms[i].left_off = ts.loff[i].empty() ? nullptr : ts.loff[i].data();
    ts.terms[i].right_off = ts.roff[i].empty() ? nullptr : ts.roff[i].data();
  }
}

}  // namespace

extern "C" {

dmrg_status dmrg_chain_create(dmrg_ctx_t ctx, int32_t L, const double* h, const double* V,
                              int32_t n_elec, int32_t two_sz, int64_t D, uint64_t seed,
                              dmrg_chain_t* out) {
  if (!out) return fail(DMRG_EINVAL, "chain_create: out is NULL");
  *out = nullptr;
  if (!h || !V || L < 2 || L > 60 || D < 1 || n_elec < 0 || n_elec > 2 * L ||
      ((n_elec + two_sz) & 1) || std::abs(two_sz) > n_elec)
    return fail(DMRG_EINVAL, "chain_create: bad arguments");
  std::unique_ptr<dmrg_chain_s> c(new (std::nothrow) dmrg_chain_s);
  if (!c) return fail(DMRG_ENOMEM, "chain_create: out of host memory");
  c->ctx = ctx;
  c->L = L;
  c->n_elec = n_elec;
  c->two_sz = two_sz;
  c->D = D;
  c->rng.seed(seed);
  c->H = hamiltonian(L, h, V);
  c->left.assign(L + 1, Block());
  c->right.assign(L + 1, Block());
  c->left[0] = empty_block();
  c->right[L] = empty_block();
  // initial right blocks: random isometries onto at most D states per block
  for (int j = L - 1; j >= 2; --j) {
    bool ok = true;
    Block E = grow(c.get(), c->right[j + 1], j, true, &ok);
    if (!ok) return fail(DMRG_EQN, "chain_create: missing block product");
    Basis kept;
    std::vector<int> map = prune(c.get(), E.b, j, kept);
    int64_t total = 0;
    for (int d : kept.dim) total += d;
    std::vector<std::vector<double>> U(E.b.qn.size());
    if (total > D) {
      // largest-remainder share of D, at least one state per sector when possible
      std::vector<int> k(kept.dim.size(), 0);
      std::vector<std::pair<double, int>> rem;
      int64_t used = 0;
      for (size_t i = 0; i < kept.dim.size(); ++i) {
        const double ex = (double)D * kept.dim[i] / (double)total;
        k[i] = std::min<int>(kept.dim[i], (int)ex);
        used += k[i];
        rem.push_back({-(ex - k[i]), (int)i});
      }
      std::sort(rem.begin(), rem.end());
      for (auto& r : rem) {
        if (used >= D) break;
        if (k[r.second] < kept.dim[r.second]) {
          ++k[r.second];
          ++used;
        }
      }
      Basis to;
      std::vector<int> map2(E.b.qn.size(), -1);
      for (size_t i = 0; i < E.b.qn.size(); ++i) {
        if (map[i] < 0 || k[map[i]] == 0) continue;
        map2[i] = (int)to.qn.size();
        to.qn.push_back(E.b.qn[i]);
        to.dim.push_back(k[map[i]]);
        U[i] = random_isometry(c->rng, E.b.dim[i], k[map[i]]);
      }
      if (dmrg_status st = renorm_any(ctx, E, to, map2, U, &c->right[j]); st != DMRG_OK) return st;
    } else {
      for (size_t i = 0; i < E.b.qn.size(); ++i)
        if (map[i] >= 0) U[i] = identity(E.b.dim[i]);
      if (dmrg_status st = renorm_any(ctx, E, kept, map, U, &c->right[j]); st != DMRG_OK) return st;
    }
  }
  *out = c.release();
  return DMRG_OK;
}

void dmrg_chain_destroy(dmrg_chain_t c) { delete c; }

dmrg_status dmrg_chain_grow_left(dmrg_chain_t c, int32_t l) {
  if (!c || l < 1 || l > c->L - 2) return fail(DMRG_EINVAL, "chain_grow_left: bad arguments");
  for (int j = 0; j < l; ++j) {
    if (c->left[j].b.qn.empty()) return fail(DMRG_EINVAL, "chain_grow_left: block not built");
    bool ok = true;
    Block E = grow(c, c->left[j], j, false, &ok);
    if (!ok) return fail(DMRG_EQN, "chain_grow_left: missing block product");
    Basis kept;
    std::vector<int> map = prune(c, E.b, c->L - j - 1, kept);
    std::vector<std::vector<double>> U(E.b.qn.size());
    for (size_t i = 0; i < E.b.qn.size(); ++i)
      if (map[i] >= 0) U[i] = identity(E.b.dim[i]);
    if (dmrg_status st = renorm_any(c->ctx, E, kept, map, U, &c->left[j + 1]); st != DMRG_OK) return st;
  }
  return DMRG_OK;
}

dmrg_status dmrg_chain_export(dmrg_chain_t c, int32_t l, int32_t* n_left, int32_t* n_right,
                              int64_t* n_terms, int64_t* lpool_len, int64_t* rpool_len, int32_t* lqn,
                              int64_t* ldim, int32_t* rqn, int64_t* rdim, int32_t* term_info,
                              int64_t* left_off, int64_t* right_off, double* lpool, double* rpool) {
  if (!c || !n_left || !n_right || !n_terms || !lpool_len || !rpool_len || l < 0 || l > c->L - 2)
    return fail(DMRG_EINVAL, "chain_export: bad arguments");
  if (c->left[l].b.qn.empty() || c->right[l + 2].b.qn.empty())
    return fail(DMRG_EINVAL, "chain_export: block not built (sweep order)");
  bool ok = true;
  Block Le = grow(c, c->left[l], l, false, &ok);
  Block Re = grow(c, c->right[l + 2], l + 1, true, &ok);
  if (!ok) return fail(DMRG_EQN, "chain_export: missing block product");
  TwoSite ts;
  assemble(c, Le, Re, ts);
  const bool fill = lqn && ldim && rqn && rdim && term_info && left_off && right_off && lpool && rpool;
  if (fill && (*n_left != (int32_t)ts.Lb.qn.size() || *n_right != (int32_t)ts.Rb.qn.size() ||
               *n_terms != (int64_t)ts.terms.size() || *lpool_len != (int64_t)ts.lpool.size() ||
               *rpool_len != (int64_t)ts.rpool.size()))
    return fail(DMRG_EINVAL, "chain_export: array sizes do not match the counts");
  *n_left = (int32_t)ts.Lb.qn.size();
  *n_right = (int32_t)ts.Rb.qn.size();
  *n_terms = (int64_t)ts.terms.size();
  *lpool_len = (int64_t)ts.lpool.size();
  *rpool_len = (int64_t)ts.rpool.size();
  if (!fill) return DMRG_OK;
  const int nl = *n_left, nr = *n_right;
  for (int i = 0; i < nl; ++i) {
    lqn[2 * i] = ts.Lb.qn[i].n;
    lqn[2 * i + 1] = ts.Lb.qn[i].s;
    ldim[i] = ts.Lb.dim[i];
  }
  for (int i = 0; i < nr; ++i) {
    rqn[2 * i] = ts.Rb.qn[i].n;
    rqn[2 * i + 1] = ts.Rb.qn[i].s;
    rdim[i] = ts.Rb.dim[i];
  }
  for (size_t t = 0; t < ts.terms.size(); ++t) {
    term_info[4 * t] = ts.terms[t].dq[0];
    term_info[4 * t + 1] = ts.terms[t].dq[1];
    term_info[4 * t + 2] = ts.terms[t].odd;
    term_info[4 * t + 3] = ts.terms[t].one_sided;
    for (int i = 0; i < nl; ++i) left_off[t * nl + i] = ts.loff[t].empty() ? -1 : ts.loff[t][i];
    for (int i = 0; i < nr; ++i) right_off[t * nr + i] = ts.roff[t].empty() ? -1 : ts.roff[t][i];
  }
  std::copy(ts.lpool.begin(), ts.lpool.end(), lpool);
  std::copy(ts.rpool.begin(), ts.rpool.end(), rpool);
  return DMRG_OK;
}

dmrg_status dmrg_chain_step(dmrg_chain_t c, int32_t l, int32_t dir, const dmrg_dav_opts* opts,
                            double* energy, double* trunc_err, dmrg_dav_result* res) {
  if (!c || !c->ctx || !opts || !energy || !trunc_err || !res || l < 0 || l > c->L - 2 ||
      (dir != 1 && dir != -1))
    return fail(DMRG_EINVAL, "chain_step: bad arguments");
  if (c->left[l].b.qn.empty() || c->right[l + 2].b.qn.empty())
    return fail(DMRG_EINVAL, "chain_step: block not built (sweep order)");
  bool ok = true;
  Block Le = grow(c, c->left[l], l, false, &ok);
  Block Re = grow(c, c->right[l + 2], l + 1, true, &ok);
  if (!ok) return fail(DMRG_EQN, "chain_step: missing block product");
  TwoSite ts;
  assemble(c, Le, Re, ts);
  std::vector<int32_t> lq, rq;
  std::vector<int64_t> ld, rd;
  for (size_t i = 0; i < ts.Lb.qn.size(); ++i) {
    lq.push_back(ts.Lb.qn[i].n);
    lq.push_back(ts.Lb.qn[i].s);
    ld.push_back(ts.Lb.dim[i]);
  }
  for (size_t i = 0; i < ts.Rb.qn.size(); ++i) {
    rq.push_back(ts.Rb.qn[i].n);
    rq.push_back(ts.Rb.qn[i].s);
    rd.push_back(ts.Rb.dim[i]);
  }
  const int32_t Q[2] = {c->n_elec, c->two_sz};
  dmrg_basis_t LB = nullptr, RB = nullptr;
  dmrg_heff_t H = nullptr;
  double *dl = nullptr, *dr = nullptr, *psi = nullptr, *U = nullptr, *S = nullptr, *Vt = nullptr;
  auto cleanup = [&]() {
    if (H) dmrg_heff_destroy(H);
    dmrg_basis_destroy(LB);
    dmrg_basis_destroy(RB);
    for (double* p : {dl, dr, psi, U, S, Vt})
      if (p) (void)hipFree(p);
  };
  dmrg_status st = dmrg_basis_create(c->ctx, (int32_t)ld.size(), lq.data(), ld.data(), &LB);
  if (st == DMRG_OK) st = dmrg_basis_create(c->ctx, (int32_t)rd.size(), rq.data(), rd.data(), &RB);
  int64_t nblk = 0, size = 0;
  if (st == DMRG_OK) st = dmrg_wfn_layout(LB, RB, Q, &nblk, nullptr, &size);
  if (st == DMRG_OK && size < 1) st = fail(DMRG_EQN, "chain_step: empty two-site space");
  const size_t lbytes = std::max<size_t>(ts.lpool.size(), 1) * 8, rbytes = std::max<size_t>(ts.rpool.size(), 1) * 8;
  if (st == DMRG_OK && (hipMalloc(&dl, lbytes) != hipSuccess || hipMalloc(&dr, rbytes) != hipSuccess ||
                        hipMalloc(&psi, size * 8) != hipSuccess))
    st = fail(DMRG_ENOMEM, "chain_step: device allocation failed");
  if (st == DMRG_OK && !ts.lpool.empty() &&
      hipMemcpy(dl, ts.lpool.data(), ts.lpool.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    st = fail(DMRG_EHIP, "chain_step: copy failed");
  if (st == DMRG_OK && !ts.rpool.empty() &&
      hipMemcpy(dr, ts.rpool.data(), ts.rpool.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    st = fail(DMRG_EHIP, "chain_step: copy failed");
  if (st == DMRG_OK)
    st = dmrg_heff_create(c->ctx, LB, RB, Q, (int64_t)ts.terms.size(), ts.terms.data(), dl,
                          (int64_t)ts.lpool.size(), dr, (int64_t)ts.rpool.size(), DMRG_FP64, &H);
  if (st == DMRG_OK) {
    // seeded random start: overlaps every eigenvector, whatever its spin
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> x0(size);
    for (auto& v : x0) v = nd(c->rng);
    if (hipMemcpy(psi, x0.data(), size * 8, hipMemcpyHostToDevice) != hipSuccess)
      st = fail(DMRG_EHIP, "chain_step: copy failed");
  }
  if (st == DMRG_OK) {
    dmrg_dav_opts o = *opts;
    o.start = 0;
    st = dmrg_davidson(H, psi, &o, res);
    if (st == DMRG_ENOCONV) st = DMRG_OK;  // reported through res->converged
  }
  *energy = res->energy;
  // truncation to D states and the renormalised block for the next step
  std::vector<int64_t> kept(ld.size(), 0);
  if (st == DMRG_OK) {
    int64_t ucap = 0, scap = 0, vcap = 0;
    for (size_t a = 0; a < ld.size(); ++a) {
      const int cidx = RB->find(Q[0] - lq[2 * a], Q[1] - lq[2 * a + 1]);
      if (cidx < 0) continue;
      const int64_t k = std::min<int64_t>(ld[a], rd[cidx]);
      ucap += ld[a] * k;
      scap += k;
      vcap += k * rd[cidx];
    }
    if (hipMalloc(&U, std::max<int64_t>(ucap, 1) * 8) != hipSuccess ||
        hipMalloc(&S, std::max<int64_t>(scap, 1) * 8) != hipSuccess ||
        hipMalloc(&Vt, std::max<int64_t>(vcap, 1) * 8) != hipSuccess)
      st = fail(DMRG_ENOMEM, "chain_step: device allocation failed");
    if (st == DMRG_OK)
      st = dmrg_svd_truncate(c->ctx, LB, RB, Q, psi, c->D, 0.0, kept.data(), U, ucap, S, scap, Vt,
                             vcap, trunc_err);
    if (st == DMRG_OK) {
      std::vector<double> hu(ucap), hv(vcap);
      if (ucap && hipMemcpy(hu.data(), U, ucap * 8, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(DMRG_EHIP, "chain_step: copy failed");
      if (st == DMRG_OK && vcap && hipMemcpy(hv.data(), Vt, vcap * 8, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(DMRG_EHIP, "chain_step: copy failed");
      if (st == DMRG_OK) {
        // unpack the kept factors per sector, in left-sector order
        std::vector<std::vector<double>> UL(Le.b.qn.size()), WR(Re.b.qn.size());
        Basis toL, toR;
        std::vector<int> mapL(Le.b.qn.size(), -1), mapR(Re.b.qn.size(), -1);
        int64_t uo = 0, vo = 0;
        for (size_t a = 0; a < ld.size(); ++a) {
          const int64_t k = kept[a];
          if (k == 0) continue;
          const int cidx = RB->find(Q[0] - lq[2 * a], Q[1] - lq[2 * a + 1]);
          const int64_t m = ld[a], n = rd[cidx];
          UL[a].assign(hu.begin() + uo, hu.begin() + uo + m * k);
          WR[cidx].assign((size_t)n * k, 0.0);  // V = Vt^T: n x k
          for (int64_t j = 0; j < k; ++j)
            for (int64_t r = 0; r < n; ++r) WR[cidx][(size_t)r * k + j] = hv[vo + j * n + r];
          uo += m * k;
          vo += k * n;
          mapL[a] = (int)toL.qn.size();
          toL.qn.push_back(Le.b.qn[a]);
          toL.dim.push_back((int)k);
        }
        for (size_t r = 0; r < Re.b.qn.size(); ++r)
          if (!WR[r].empty()) {
            mapR[r] = (int)toR.qn.size();
            toR.qn.push_back(Re.b.qn[r]);
            toR.dim.push_back((int)(WR[r].size() / Re.b.dim[r]));
          }
        if (dir == 1)
          st = renorm_any(c->ctx, Le, toL, mapL, UL, &c->left[l + 1]);
        else
          st = renorm_any(c->ctx, Re, toR, mapR, WR, &c->right[l + 1]);
      }
    }
  }
  cleanup();
  return st;
}

}  // extern "C"

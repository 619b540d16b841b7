// Truncating SVD of the two-site wavefunction (after the Davidson solve).
//
// The paper factorises the optimised tensor and keeps D states
// (Introduction: "matrix factorization"; Numerical procedure: D sets the
// accuracy).  With U(1)xU(1) symmetry the wavefunction is block diagonal in
// the enlarged-left sector, so every block Psi[q, Q-q] is decomposed on its
// own by one-sided (Hestenes) Jacobi on the block's columns (or on its
// transpose when it is wide).  Every launch is one round of a round-robin
// ordering for all blocks together, one wavefront per disjoint column pair,
// so the largest blocks are spread over the whole GPU; sweeps repeat until
// no block rotates.  The
// singular values of all blocks are then pooled and truncated on the host
// (global top-D with a deterministic tie-break), and a pack kernel writes the
// kept factors.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace dmrg {

// Sweeps after which a block that still rotates is reported as not
// converged (DMRG_ENOCONV).  Quadratic convergence makes the usual count
// about ten; decaying spectra spanning the whole FP64 range need more.
constexpr int SVD_MAX_SWEEPS = 80;

struct SvdBlock {
  int64_t src;    // offset of the block in psi (row-major m x n)
  int64_t boff;   // work: B, column-major r x c (r >= c)
  int64_t voff;   // work: V, column-major c x c
  int64_t soff;   // sigma offset
  int32_t m, n;   // block shape
  int32_t r, c;   // shape of B (B = X if n <= m, else X^T)
  int32_t trans;  // 1 when B = X^T
  int32_t pad;
};

struct PackBlock {
  int64_t uoff, soff_out, vtoff;  // output offsets
  int64_t perm;                   // offset of this block's permutation
  int32_t k;                      // kept values
  int32_t pad;
};

__global__ __launch_bounds__(256) void svd_load_kernel(const SvdBlock* __restrict__ blocks,
                                                       const double* __restrict__ psi,
                                                       double* __restrict__ work) {
  const SvdBlock b = blocks[blockIdx.x];
  const double* X = psi + b.src;
  double* B = work + b.boff;
  double* V = work + b.voff;
  const int64_t mn = (int64_t)b.m * b.n;
  for (int64_t e = threadIdx.x; e < mn; e += blockDim.x) {
    const int i = (int)(e / b.n), j = (int)(e % b.n);  // X[i][j]
    if (!b.trans)
      B[(int64_t)j * b.m + i] = X[e];  // column j of X
    else
      B[(int64_t)i * b.n + j] = X[e];  // column i of X^T is row i of X
  }
  for (int64_t e = threadIdx.x; e < (int64_t)b.c * b.c; e += blockDim.x)
    V[e] = (e / b.c == e % b.c) ? 1.0 : 0.0;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Column pair slot `pi` of round `rd` in the round-robin ordering of m (even)
// columns: every round pairs all columns disjointly, m - 1 rounds visit every
// pair once (a sweep).
__device__ __forceinline__ void rr_pair(int pi, int rd, int m, int* p, int* q) {
  int a = pi == 0 ? 0 : 1 + (pi - 1 + rd) % (m - 1);
  const int pos = m - 1 - pi;
  int b = pos == 0 ? 0 : 1 + (pos - 1 + rd) % (m - 1);
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

struct SvdPair {
  int32_t blk, pi;  // block and pair slot
};

// One round of one-sided (Hestenes) Jacobi over every block at once: one
// wavefront per column pair; the pairs of a round are disjoint, so the
// rotations of a launch commute and the result does not depend on how waves
// are scheduled.  A pair rotates when its columns are not orthogonal to
// relative tolerance eps * sqrt(r) (r the column length: the rounding level
// of a computed inner product, the usual one-sided Jacobi criterion); V
// accumulates the rotations; flags[blk] records that the block rotated in
// this sweep.  Rotation of the 2x2 Gram matrix [[alpha, gamma], [gamma, beta]]
// by the standard formulas.
__global__ __launch_bounds__(256) void svd_round_kernel(const SvdBlock* __restrict__ blocks,
                                                        const SvdPair* __restrict__ pairs,
                                                        int64_t npairs, int rd,
                                                        double* __restrict__ work,
                                                        int32_t* __restrict__ flags, double eps) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (wid >= npairs) return;
  const SvdPair pr = pairs[wid];
  const SvdBlock b = blocks[pr.blk];
  const int r = b.r, c = b.c;
  const int m = c + (c & 1);
  if (c < 2 || rd >= m - 1) return;
  int p, q;
  rr_pair(pr.pi, rd, m, &p, &q);
  if (q >= c) return;  // bye
  double* B = work + b.boff;
  double* V = work + b.voff;
  double* bp = B + (int64_t)p * r;
  double* bq = B + (int64_t)q * r;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = lane; i < r; i += 64) {
    const double x = bp[i], y = bq[i];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  if (!(fabs(ga) > eps * sqrt((double)r) * sqrt(al * be)) || ga == 0.0) return;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  for (int i = lane; i < r; i += 64) {
    const double x = bp[i], y = bq[i];
    bp[i] = cs * x - sn * y;
    bq[i] = sn * x + cs * y;
  }
  double* vp = V + (int64_t)p * c;
  double* vq = V + (int64_t)q * c;
  for (int i = lane; i < c; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = cs * x - sn * y;
    vq[i] = sn * x + cs * y;
  }
  if (lane == 0) flags[pr.blk] = 1;
}

__global__ void svd_clear_kernel(int32_t* __restrict__ flags, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) flags[i] = 0;
}

// Singular values = column norms of the converged B; its columns, normalised,
// are the singular vectors on B's side.
__global__ __launch_bounds__(256) void svd_finish_kernel(const SvdBlock* __restrict__ blocks,
                                                         double* __restrict__ work,
                                                         double* __restrict__ sigma) {
  const SvdBlock b = blocks[blockIdx.x];
  double* B = work + b.boff;
  const int r = b.r, c = b.c;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int j = wave; j < c; j += nwaves) {
    double* bj = B + (int64_t)j * r;
    double s2 = 0.0;
    for (int i = lane; i < r; i += 64) s2 += bj[i] * bj[i];
    s2 = wave_sum(s2);
    const double s = sqrt(s2);
    if (lane == 0) sigma[b.soff + j] = s;
    if (s > 0.0) {
      const double inv = 1.0 / s;
      for (int i = lane; i < r; i += 64) bj[i] *= inv;
    }
  }
}

__global__ __launch_bounds__(256) void svd_pack_kernel(const SvdBlock* __restrict__ blocks,
                                                       const PackBlock* __restrict__ packs,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ work,
                                                       const double* __restrict__ sigma,
                                                       double* __restrict__ U, double* __restrict__ S,
                                                       double* __restrict__ Vt) {
  const SvdBlock b = blocks[blockIdx.x];
  const PackBlock pk = packs[blockIdx.x];
  if (pk.k == 0) return;
  const double* B = work + b.boff;
  const double* V = work + b.voff;
  const int32_t* pm = perm + pk.perm;
  const int k = pk.k;
  // U (m x k) row-major, Vt (k x n) row-major
  for (int64_t e = threadIdx.x; e < (int64_t)b.m * k; e += blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    const int col = pm[j];
    U[pk.uoff + e] = !b.trans ? B[(int64_t)col * b.r + i] : V[(int64_t)col * b.c + i];
  }
  for (int64_t e = threadIdx.x; e < (int64_t)k * b.n; e += blockDim.x) {
    const int j = (int)(e / b.n), l = (int)(e % b.n);
    const int col = pm[j];
    Vt[pk.vtoff + e] = !b.trans ? V[(int64_t)col * b.c + l] : B[(int64_t)col * b.r + l];
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) S[pk.soff_out + j] = sigma[b.soff + pm[j]];
}

}  // namespace dmrg

using namespace dmrg;

namespace dmrg {

// Device temporaries of one truncation, carved out of one arena (aligned to
// 256 bytes each): the working copies B and V, the block and pair tables,
// the singular values, the rotation flags, the pack table and the kept
// permutation (at most one entry per singular value).
struct SvdArena {
  size_t work, blocks, sig, pairs, flags, packs, perm, total;
};

SvdArena svd_arena(int64_t woff, int nb, int64_t soff, int64_t npairs) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  SvdArena a{};
  size_t o = 0;
  a.work = o;   o += up(std::max<int64_t>(woff, 1) * sizeof(double));
  a.blocks = o; o += up((size_t)nb * sizeof(SvdBlock));
  a.sig = o;    o += up(std::max<int64_t>(soff, 1) * sizeof(double));
  a.pairs = o;  o += up(std::max<int64_t>(npairs, 1) * sizeof(SvdPair));
  a.flags = o;  o += up((size_t)nb * sizeof(int32_t));
  a.packs = o;  o += up((size_t)nb * sizeof(PackBlock));
  a.perm = o;   o += up(std::max<int64_t>(soff, 1) * sizeof(int32_t));
  a.total = o;
  return a;
}

// The truncation itself.  arena: device memory of at least arena_cap bytes
// for the temporaries, or NULL to allocate them here (one hipMalloc, freed
// before returning).
dmrg_status svd_truncate_impl(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2],
                              const double* psi, int64_t max_keep, double cutoff, int64_t* kept_dim,
                              double* U, int64_t u_cap, double* S, int64_t s_cap, double* Vt,
                              int64_t vt_cap, double* trunc_err, char* arena, size_t arena_cap,
                              const char* who) {
  const std::string name(who);
  if (!ctx || !L || !R || !Q || !psi || !kept_dim || !trunc_err || max_keep < 0 || !(cutoff >= 0.0))
    return fail(DMRG_EINVAL, name + ": bad arguments");
  hipStream_t s = ctx->stream;
  const int nL = (int)L->dim.size();
  std::vector<SvdBlock> blocks;
  std::vector<int> sector;
  int64_t off = 0, woff = 0, soff = 0;
  for (int a = 0; a < nL; ++a) {
    kept_dim[a] = 0;
    const int cidx = R->find(Q[0] - L->qn[2 * a], Q[1] - L->qn[2 * a + 1]);
    if (cidx < 0) continue;
    SvdBlock b{};
    b.src = off;
    b.m = (int32_t)L->dim[a];
    b.n = (int32_t)R->dim[cidx];
    b.trans = b.n > b.m ? 1 : 0;
    b.r = b.trans ? b.n : b.m;
    b.c = b.trans ? b.m : b.n;
    b.boff = woff;
    woff += (int64_t)b.r * b.c;
    b.voff = woff;
    woff += (int64_t)b.c * b.c;
    b.soff = soff;
    soff += b.c;
    off += (int64_t)b.m * b.n;
    blocks.push_back(b);
    sector.push_back(a);
  }
  if (blocks.empty()) return fail(DMRG_EQN, name + ": no block has total Q");
  const int nb = (int)blocks.size();
  // flattened (block, pair slot) list; rounds per sweep = the largest block's
  std::vector<SvdPair> pairs;
  int max_rounds = 0;
  for (int i = 0; i < nb; ++i) {
    const int c = blocks[i].c, m = c + (c & 1);
    if (c < 2) continue;
    for (int pi = 0; pi < m / 2; ++pi) pairs.push_back(SvdPair{i, pi});
    max_rounds = std::max(max_rounds, m - 1);
  }
  const int64_t npairs = (int64_t)pairs.size();
  const SvdArena lay = svd_arena(woff, nb, soff, npairs);
  char* mem = arena;
  if (arena) {
    if (lay.total > arena_cap)
      return fail(DMRG_ENOMEM, name + ": needs " + std::to_string(lay.total) +
                                   " bytes of device scratch, more than its " +
                                   std::to_string(arena_cap) + "-byte maximum");
  } else if (hipMalloc((void**)&mem, lay.total) != hipSuccess) {
    return fail(DMRG_ENOMEM, name + ": device allocation failed");
  }
  auto cleanup = [&]() {
    if (!arena && mem) (void)hipFree(mem);
  };
  double* work = (double*)(mem + lay.work);
  SvdBlock* dblocks = (SvdBlock*)(mem + lay.blocks);
  double* dsig = (double*)(mem + lay.sig);
  SvdPair* dpairs = (SvdPair*)(mem + lay.pairs);
  int32_t* dflags = (int32_t*)(mem + lay.flags);
  PackBlock* dpacks = (PackBlock*)(mem + lay.packs);
  int32_t* dperm = (int32_t*)(mem + lay.perm);
  std::vector<double> sig(soff);
  hipError_t e = hipMemcpyAsync(dblocks, blocks.data(), nb * sizeof(SvdBlock), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !pairs.empty())
    e = hipMemcpyAsync(dpairs, pairs.data(), pairs.size() * sizeof(SvdPair), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    svd_load_kernel<<<nb, 256, 0, s>>>(dblocks, psi, work);
    e = hipGetLastError();
  }
  const unsigned grid = (unsigned)std::max<int64_t>(1, (npairs + 3) / 4);
  std::vector<int32_t> flags(nb, 0);
  bool converged = npairs == 0;
  for (int sweep = 0; sweep < SVD_MAX_SWEEPS && !converged && e == hipSuccess; ++sweep) {
    svd_clear_kernel<<<1, 256, 0, s>>>(dflags, nb);
    for (int rd = 0; rd < max_rounds; ++rd)
      svd_round_kernel<<<grid, 256, 0, s>>>(dblocks, dpairs, npairs, rd, work, dflags, 2.220446049250313e-16);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), dflags, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) converged = std::all_of(flags.begin(), flags.end(), [](int32_t f) { return f == 0; });
  }
  if (e == hipSuccess) {
    svd_finish_kernel<<<nb, 256, 0, s>>>(dblocks, work, dsig);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(sig.data(), dsig, soff * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return fail(DMRG_EHIP, name + ": " + hipGetErrorString(e));
  }
  // per block: descending order; globally: (sigma desc, sector asc, position asc)
  std::vector<std::vector<int32_t>> order(nb);
  struct Entry {
    double s;
    int blk, pos;
  };
  std::vector<Entry> all;
  for (int i = 0; i < nb; ++i) {
    auto& o = order[i];
    o.resize(blocks[i].c);
    for (int j = 0; j < blocks[i].c; ++j) o[j] = j;
    const double* sg = sig.data() + blocks[i].soff;
    std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return sg[x] > sg[y]; });
    for (int j = 0; j < blocks[i].c; ++j) all.push_back(Entry{sg[o[j]], i, j});
  }
  std::stable_sort(all.begin(), all.end(), [](const Entry& x, const Entry& y) {
    if (x.s != y.s) return x.s > y.s;
    if (x.blk != y.blk) return x.blk < y.blk;
    return x.pos < y.pos;
  });
  std::vector<int> kept(nb, 0);
  double err = 0.0;
  int64_t nkeep = 0;
  for (const Entry& en : all) {
    if (nkeep < max_keep && en.s > cutoff) {
      kept[en.blk]++;
      ++nkeep;
    } else {
      err += en.s * en.s;
    }
  }
  *trunc_err = err;
  std::vector<PackBlock> packs(nb);
  std::vector<int32_t> perm;
  int64_t uo = 0, so = 0, vo = 0;
  for (int i = 0; i < nb; ++i) {
    PackBlock& p = packs[i];
    p.k = kept[i];
    p.uoff = uo;
    p.soff_out = so;
    p.vtoff = vo;
    p.perm = (int64_t)perm.size();
    for (int j = 0; j < kept[i]; ++j) perm.push_back(order[i][j]);
    uo += (int64_t)blocks[i].m * kept[i];
    so += kept[i];
    vo += (int64_t)kept[i] * blocks[i].n;
    kept_dim[sector[i]] = kept[i];
  }
  if ((uo > 0 && (!U || uo > u_cap)) || (so > 0 && (!S || so > s_cap)) || (vo > 0 && (!Vt || vo > vt_cap))) {
    cleanup();
    return fail(DMRG_EINVAL, name + ": output buffers too small");
  }
  e = hipMemcpyAsync(dpacks, packs.data(), nb * sizeof(PackBlock), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !perm.empty())
    e = hipMemcpyAsync(dperm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nkeep > 0) {
    svd_pack_kernel<<<nb, 256, 0, s>>>(dblocks, dpacks, dperm, work, dsig, U, S, Vt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return fail(DMRG_EHIP, name + ": " + hipGetErrorString(e));
  if (!converged)
    return fail(DMRG_ENOCONV, name + ": Jacobi sweeps still rotating after " +
                                  std::to_string(SVD_MAX_SWEEPS) + " sweeps (outputs written, not converged)");
  return DMRG_OK;
}

}  // namespace dmrg

extern "C" dmrg_status dmrg_svd_truncate(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R,
                                         const int32_t Q[2], const double* psi, int64_t max_keep,
                                         double cutoff, int64_t* kept_dim, double* U, int64_t u_cap,
                                         double* S, int64_t s_cap, double* Vt, int64_t vt_cap,
                                         double* trunc_err) {
  return svd_truncate_impl(ctx, L, R, Q, psi, max_keep, cutoff, kept_dim, U, u_cap, S, s_cap, Vt,
                           vt_cap, trunc_err, nullptr, 0, "svd_truncate");
}

// ---------------------------------------------------------------------------
// Allocation-free truncation.  Its temporaries live in `scratch`, a
// file-scope device array that every device the library runs on holds (one
// copy each) until the process ends.  In host code the array's name is not a
// device address: its per-device address comes from hipGetSymbolAddress,
// taken once per device when a context is created on it, and only that
// pointer is handed to kernels and copies.
namespace dmrg {

constexpr size_t SVD_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) char scratch[SVD_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch[MAX_DEVICES] = {};
}  // namespace

// Called by dmrg_ctx_create with `device` current.
dmrg_status svd_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(DMRG_ENOTSUP, "svd scratch: device ordinal too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return DMRG_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(DMRG_EHIP, std::string("svd scratch: hipGetSymbolAddress: ") + hipGetErrorString(e));
  g_scratch[device] = (char*)ptr;
  return DMRG_OK;
}

}  // namespace dmrg

extern "C" dmrg_status dmrg_svd_truncate_noalloc(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R,
                                                 const int32_t Q[2], const double* psi,
                                                 int64_t max_keep, double cutoff, int64_t* kept_dim,
                                                 double* U, int64_t u_cap, double* S, int64_t s_cap,
                                                 double* Vt, int64_t vt_cap, double* trunc_err) {
  if (!ctx) return fail(DMRG_EINVAL, "svd_truncate_noalloc: bad arguments");
  char* mem = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < MAX_DEVICES) mem = g_scratch[ctx->device];
  }
  if (!mem) return fail(DMRG_EINVAL, "svd_truncate_noalloc: no scratch address for the context's device");
  return svd_truncate_impl(ctx, L, R, Q, psi, max_keep, cutoff, kept_dim, U, u_cap, S, s_cap, Vt,
                           vt_cap, trunc_err, mem, SVD_SCRATCH_BYTES, "svd_truncate_noalloc");
}

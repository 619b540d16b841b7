// FP64 output tile of the grouped GEMM with operands staged straight into LDS
// (buffer-to-LDS loads, no register staging) through an NST-deep ring of K
// tiles.  Shared by the per-phase kernels and the persistent matvec kernel.
//
// Work description as in internal.h: a problem C (M x N) = [beta ? C : 0] +
// sum over its segments of alpha * X (M x K) * Z (K x N), operands named by
// buffer id and offset, either stored K-contiguous (row-major in K) or
// row-contiguous.  Every element's sum runs in the same order as in the
// register-staged kernel: segments in order, 16-deep K tiles, four K values
// per v_mfma_f64_16x16x4f64 step, alpha applied to the X value before the
// product, zeros past the end of K.  The results are therefore bit-identical.
//
// LDS image of one K tile (16 K values), per operand, in 16-byte chunks of two
// doubles; lane l of a load writes chunk (base + l), so the layout is chosen by
// which global chunk each lane fetches:
//   K-contiguous operand:  element (r, k) at double r*16 + 2*((k>>1) ^ ((r>>1)&7)) + (k&1)
//   row-contiguous operand: element (r, k) at double k*ROWS + (r ^ ((k&1) << 4))
// The XOR terms spread the 16 rows x 4 K values that one fragment read
// touches over distinct LDS banks.
//
// Values past the end of a segment's K read as zero: chunks that start past K
// are loaded with an out-of-range offset (the buffer range check returns
// zeros), and the second value of a K-contiguous chunk that straddles K is
// zeroed in LDS before the tile is used.  Every load is bounded by the end of
// its buffer.
#pragma once

#include <type_traits>

#include "internal.h"

namespace dmrg {
namespace dma {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr uint32_t OOB = 0xffffffffu;
constexpr int BK = 16;

// Buffer resource over [p, p + bytes_left): loads at or past the end read as
// zero instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double* p, uint64_t bytes_left) {
  const uint32_t n = bytes_left > 0x7fffffffull ? 0x7fffffffu : (uint32_t)bytes_left;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, (int)n, 0x00020000);
}

// s_waitcnt vmcnt(N) leaving the other counters alone (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Issue side of one operand: the global chunks this thread fetches for every
// K tile of the current segment.
template <int ROWS, int NT>
struct Issue {
  static constexpr int NI = ROWS * BK / 2 / NT;  // chunks per thread per K tile
  static_assert(ROWS * BK / 2 % NT == 0 && NI >= 1, "chunk split");
  static_assert(ROWS >= 32 && ROWS % 32 == 0, "row-contiguous swizzle needs 16+ chunks per K row");
  const double* base;  // uniform: row r0 of the block at the current k0
  const double* end;   // uniform: end of the operand's buffer
  int64_t kstep;       // uniform: elements between K tiles
  uint32_t off[NI];    // per thread: byte offset of each chunk from base
  int kq[NI];          // per thread: K index (within the tile) of the chunk's first value

  __device__ __forceinline__ void setup(const double* blk, const double* buf_end, int ld, bool kc,
                                        int r0, int nrows, int tid) {
    end = buf_end;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int p = j * NT + tid;
      if (kc) {
        const int r = p >> 3;
        const int kk = 2 * ((p & 7) ^ ((r >> 1) & 7));
        off[j] = r0 + r < nrows ? (uint32_t)(r * ld + kk) * 8u : OOB;
        kq[j] = kk;
      } else {
        const int k = p / (ROWS / 2);
        const int r = 2 * ((p % (ROWS / 2)) ^ ((k & 1) << 3));
        off[j] = r0 + r < nrows ? (uint32_t)(k * ld + r) * 8u : OOB;
        kq[j] = k;
      }
    }
    base = kc ? blk + (int64_t)r0 * ld : blk + r0;
    kstep = kc ? BK : (int64_t)BK * ld;
  }

  // Loads of the current K tile into the stage at `dst` (uniform LDS
  // address); kleft values remain in the segment: chunks that start at or
  // past K read as zero.
  __device__ __forceinline__ void issue(double* dst, int wave, int kleft) const {
    const __amdgpu_buffer_rsrc_t rs = rsrc(base, (uint64_t)(end - base) * 8u);
#pragma unroll
    for (int j = 0; j < NI; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + 2 * (j * NT + wave * 64)), 16,
                                               kq[j] < kleft ? off[j] : OOB, 0, 0, 0);
  }

  __device__ __forceinline__ void advance() { base += kstep; }
};

// A K-contiguous chunk whose second value lies past K (odd kleft) holds the
// next row's value there: zero it once the tile has landed.  Each thread
// fixes the chunks it loaded (their positions do not depend on the segment).
template <int ROWS, int NT>
__device__ __forceinline__ void fix_tail(double* dst, int kleft, int tid) {
  constexpr int NI = ROWS * BK / 2 / NT;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int p = j * NT + tid;
    const int r = p >> 3;
    const int kk = 2 * ((p & 7) ^ ((r >> 1) & 7));
    if (kk + 1 == kleft) dst[2 * p + 1] = 0.0;
  }
}

// Read side: byte offset of fragment i at K step s within an operand's
// stage, for either layout (both kept; the stage's layout selects):
//   K-contiguous operand:  ua[s] + 2048 i      (ua per lane)
//   row-contiguous operand: vb[i] + 32 s ROWS  (vb per lane)
template <int ROWS, int F>
struct Reader {
  uint32_t ua[4], vb[F];
  __device__ __forceinline__ void setup(int rbase, int fr, int fk) {
    // (k >> 1) ^ ((row >> 1) & 7) with k = 4s + fk, row = rbase + 16i + fr
    // (rbase a multiple of 16) is (2s + (fk >> 1)) ^ (fr >> 1)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      ua[s] = 8u * ((rbase + fr) * 16 + ((((2 * s + (fk >> 1)) ^ (fr >> 1)) << 1) | (fk & 1)));
#pragma unroll
    for (int i = 0; i < F; ++i) vb[i] = 8u * (fk * ROWS + ((rbase + 16 * i) ^ ((fk & 1) << 4)) + fr);
  }
  __device__ __forceinline__ uint32_t at(bool kc, int s, int i) const {
    return kc ? ua[s] + 2048u * i : vb[i] + 32u * s * ROWS;
  }
};

// One output tile (tm, tn) of problem p.  lds: NST * (BM + BN) * BK doubles
// (16-byte aligned).  rot rotates the wave roles (spreads the idle waves of
// edge tiles over the SIMDs).
template <int BM, int BN, int WGM, int WGN, int NST>
__device__ __forceinline__ void tile_f64(const Bases& bases, const Prob& p, const Seg* __restrict__ segs,
                                         int tm, int tn, int rot, double* lds) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN, FM = WM / 16, FN = WN / 16;
  constexpr int XS = BM * BK, STAGE = (BM + BN) * BK;
  static_assert(FM >= 1 && FN >= 1 && NST >= 2 && NST <= 3, "tile shape");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int wm, wn;
  if (WGM == 2 && WGN == 4) {
    const int simd = (wave + rot) & 3, slot = wave >> 2;
    wm = slot;
    wn = slot == 0 ? simd : (simd + 2) & 3;
  } else {
    const int role = (wave + 2 * rot) % NW;
    wm = role / WGN;
    wn = role % WGN;
  }
  const int m0 = tm * BM, n0 = tn * BN;
  const int fr = lane & 15, fk = lane >> 4;
  const bool active = m0 + wm * WM < p.M && n0 + wn * WN < p.N;

  d4 acc[FM][FN];
  double* __restrict__ C = bases.p[p.cbuf] + p.coff;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (p.beta) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = min(m0 + wm * WM + i * 16 + fk + 4 * v, p.M - 1);
          const int n = min(n0 + wn * WN + j * 16 + fr, p.N - 1);
          acc[i][j][v] = C[(int64_t)m * p.ldc + n];
        }
  }

  if (p.nseg > 0) {
    Issue<BM, NT> xi;
    Issue<BN, NT> zi;
    Reader<BM, FM> xr;
    Reader<BN, FN> zr;
    const int s_end = p.seg0 + p.nseg;
    int s = p.seg0, k0 = 0;
    Seg g = segs[s];
    auto setup = [&]() {
      xi.setup(bases.p[g.xbuf] + g.xoff, bases.p[g.xbuf] + bases.len[g.xbuf], g.ldx, !g.xt, m0, p.M, tid);
      zi.setup(bases.p[g.zbuf] + g.zoff, bases.p[g.zbuf] + bases.len[g.zbuf], g.ldz, g.zt, n0, p.N, tid);
    };
    setup();
    // per-stage metadata of the K tile it holds (uniform)
    double st_alpha[NST];
    int st_kleft[NST], st_lay[NST];
    xr.setup(wm * WM, fr, fk);
    zr.setup(wn * WN, fr, fk);
    bool more = true;
    // issue the current cursor's K tile into stage st and advance the cursor
    auto issue = [&](int st) {
      st_alpha[st] = g.alpha;
      st_kleft[st] = g.K - k0;
      st_lay[st] = (g.xt ? 0 : 1) | (g.zt ? 2 : 0);
      xi.issue(lds + st * STAGE, wave, g.K - k0);
      zi.issue(lds + st * STAGE + XS, wave, g.K - k0);
      k0 += BK;
      if (k0 >= g.K) {
        ++s;
        k0 = 0;
        if (s < s_end) {
          g = segs[s];
          setup();
        } else {
          more = false;
        }
      } else {
        xi.advance();
        zi.advance();
      }
    };
    // MFMAs of one stage.  The X values are multiplied by alpha (exact when
    // alpha is 1).
    auto compute = [&](int st) {
      if (!active) return;
      const int lay = st_lay[st];
      const bool xkc = lay & 1, zkc = (lay >> 1) & 1;
      const char* X = (const char*)(lds + st * STAGE);
      const char* Z = X + XS * 8;
      const double al = st_alpha[st];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        double a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = al * *(const double*)(X + xr.at(xkc, ks, i));
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = *(const double*)(Z + zr.at(zkc, ks, j));
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    };
    constexpr int OPS = Issue<BM, NT>::NI + Issue<BN, NT>::NI;  // loads per K tile per thread
    // prologue: NST - 1 K tiles in flight
    int filled = 0;
#pragma unroll
    for (int st = 0; st < NST - 1; ++st)
      if (more) {
        issue(st);
        ++filled;
      }
    int st = 0;
    while (true) {
      // the tile of stage st has landed once at most (filled - 1) later tiles'
      // loads are outstanding
      if (NST == 3 && filled >= 2)
        wait_vm<OPS>();
      else
        wait_vm<0>();
      if ((st_kleft[st] & 1) && st_kleft[st] < BK) {
        if (st_lay[st] & 1) fix_tail<BM, NT>(lds + st * STAGE, st_kleft[st], tid);
        if (st_lay[st] & 2) fix_tail<BN, NT>(lds + st * STAGE + XS, st_kleft[st], tid);
      }
      __syncthreads();
      const int nxt = st == 0 ? NST - 1 : st - 1;  // the stage consumed last round
      if (more) {
        issue(nxt);
        ++filled;
      }
      compute(st);
      --filled;
      if (filled == 0) break;
      st = st + 1 == NST ? 0 : st + 1;
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * WM + i * 16 + fk + 4 * v;
        const int n = n0 + wn * WN + j * 16 + fr;
        if (m < p.M && n < p.N) C[(int64_t)m * p.ldc + n] = acc[i][j][v];
      }
}

}  // namespace dma
}  // namespace dmrg

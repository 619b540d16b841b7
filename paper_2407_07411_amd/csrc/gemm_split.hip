// Split-precision grouped GEMM: FP64 operands as three BF16 slices on the
// gfx950 BF16 matrix cores, FP32 accumulation over a few K tiles, FP64
// combine.
//
// Each FP64 operand value a is split while it is staged into LDS:
// f = fp32(a), a0 = bf16(f), a1 = bf16(f - a0), a2 = bf16(f - a0 - a1); the
// differences are exact in FP32, so a = a0 + a1 + a2 + O(2^-24 |a|).  The
// product of two split values keeps the six slice products with i + j <= 2
// (the dropped ones are O(2^-24) relative).  Slice products are exact in FP32
// and the matrix cores sum them in FP32.  Two accumulation forms: the FP32
// partial, times the segment's alpha, is added into an FP64 accumulator at
// the end of every segment and every SPLIT_FLUSH_K values of K (FP32
// rounding spans at most SPLIT_FLUSH_K values); or, for the 128 x 128 tiles
// by default, alpha multiplies the operator operand while it is staged, the
// FP32 accumulators hold the whole sum, and the plan cuts split-precision
// sums at SPLIT_ACC32_KCHUNK values, whose parts the ordered reduction adds
// in FP64.  The second form frees the FP64 accumulators' registers, so two
// workgroups share a CU.  The problem/segment/tile tables and the
// output-stationary ordering are those of the FP64 kernel, so results are
// deterministic.
//
// Staging: a thread owns groups of 8 K values of one operand row (one row of X
// or one column of Z).  With KG = BK/8 groups per row and K tile, group kg
// holds k = k0 + kg + KG e, e = 0..7, at LDS positions 8kg + e; X and Z use
// the same K permutation, so the products are unchanged.  Where the operand
// is contiguous in K, KG neighbouring lanes read one run of KG doubles per
// load; where it is contiguous in the row index, neighbouring lanes read
// neighbouring rows.  The eight values are converted pairwise
// (v_cvt_pk_bf16_f32) and each slice lands in LDS as one 16-byte store.  With
// two LDS buffers the split and store of the next K tile run while the matrix
// cores work on the current one and one barrier separates K tiles; with one
// buffer (deeper K tiles) two barriers do.
//
// Pre-split operands: the vector and the intermediates of the two-GEMM chains
// can be held as packed words (three BF16 slices of one value per 64-bit
// word, made by the same split), written once by the kernel that produces
// them; staging such an operand only moves the slices into place.  Operator
// blocks stay FP64 and are split while staged.  Both forms give the same
// slices, so the results are bit-identical.
//
// Matrix core: v_mfma_f32_32x32x16_bf16.  Lanes: A[i][k] holds i = l%32,
// k = 8(l/32) + e; B[k][j] holds j = l%32, k = 8(l/32) + e (e = 0..7); the 16
// result floats of lane l are D[8(v/4) + 4(l/32) + v%4][l%32] (measured).
#include <cstdlib>

#include "internal.h"

namespace dmrg {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

constexpr int SPLIT_BK = 32;            // default K tile depth
constexpr int SPLIT_FLUSH_K = 128;      // K values per FP32 partial

__device__ __forceinline__ int64_t xcd_remap_s(int64_t bid, int64_t n) {
  const int64_t per = n / 8, rem = n % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ uint32_t pk_bits(bf2 h) { return __builtin_bit_cast(uint32_t, h); }

// Split two FP64 values into three packed BF16 pairs.
__device__ __forceinline__ void split_pair(double a, double b, uint32_t& s0, uint32_t& s1,
                                           uint32_t& s2) {
  const f2v f = {(float)a, (float)b};
  const bf2 h0 = __builtin_convertvector(f, bf2);
  const f2v r1 = f - __builtin_convertvector(h0, f2v);
  const bf2 h1 = __builtin_convertvector(r1, bf2);
  const f2v r2 = r1 - __builtin_convertvector(h1, f2v);
  const bf2 h2 = __builtin_convertvector(r2, bf2);
  s0 = pk_bits(h0);
  s1 = pk_bits(h1);
  s2 = pk_bits(h2);
}

// Packed word of one value from its slices (low, high halves of the pairs
// made by split_pair: half 0 is the pair's first value).
__device__ __forceinline__ uint64_t pack_word(uint32_t s0, uint32_t s1, uint32_t s2, int half) {
  const uint32_t a0 = half ? s0 >> 16 : s0 & 0xffffu;
  const uint32_t a1 = half ? s1 >> 16 : s1 & 0xffffu;
  const uint32_t a2 = half ? s2 >> 16 : s2 & 0xffffu;
  return (uint64_t)(a0 | (a1 << 16)) | ((uint64_t)a2 << 32);
}

__global__ __launch_bounds__(256) void pack_split_kernel(const double* __restrict__ x,
                                                          uint64_t* __restrict__ out, int64_t n) {
  const int64_t np = (n + 1) / 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = 2 * i;
    const bool two = j + 1 < n;
    uint32_t s0, s1, s2;
    split_pair(x[j], two ? x[j + 1] : 0.0, s0, s1, s2);
    out[j] = pack_word(s0, s1, s2, 0);
    if (two) out[j + 1] = pack_word(s0, s1, s2, 1);
  }
}

dmrg_status launch_pack_split(const double* x, double* out, int64_t n, hipStream_t s) {
  if (n <= 0) return DMRG_OK;
  const int64_t np = (n + 1) / 2;
  const int64_t blocks = std::min<int64_t>((np + 255) / 256, 2048);
  pack_split_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, reinterpret_cast<uint64_t*>(out), n);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}


// The 128 x 128 split kernel: the FP32-accumulating one with eight 32 x 64
// waves in a 61 KB buffer (two workgroups per CU, one staging while the
// other multiplies) by default; DMRG_HEFF_SPLIT_ACC32 = 0 selects the
// FP64-accumulating sixteen-wave kernel.  Read once per process.  A/B on the
// D=4096 matvec (split precision, whole matvec): FP64-accumulating 401 ms,
// ||dy||/||y|| 2.2e-7; FP32-accumulating with sums cut at 1024 / 2048 / 4096:
// 370 / 355 / 355 ms, 5.9e-7 / 8.6e-7 / 1.3e-6 (the cut adds ordered FP64
// reductions); the same with sixteen 32 x 32 waves and 64-deep tiles (one
// workgroup per CU): 415 ms; eight 64 x 32 waves: as 32 x 64; two 32-deep
// buffers (one workgroup per CU): 444 ms.
int split_acc32_variant() {
  static const int v = [] {
    const char* e = std::getenv("DMRG_HEFF_SPLIT_ACC32");
    return e ? std::atoi(e) : 2;
  }();
  return v;
}

// The 8-value groups of one operand (ROWS x BK per K tile) that a thread
// stages: up to G groups, group r is gi = tid + r * NT < ROWS * KG.  The
// slice planes hold the tile in natural K order, and the assignment follows
// the operand's layout so that every load instruction is coalesced:
// * contiguous in the row index (element (row, k) at base + k*ld + row): a
//   group is one row at 8 consecutive k, consecutive lanes take consecutive
//   rows; each value is one 8-byte load, the group's slices one 16-byte LDS
//   store each;
// * contiguous in K (base + row*ld + k): a group is one K pair (2 consecutive
//   k) in 4 rows ROWS/4 apart, consecutive lanes take consecutive pairs of a
//   row (16 lanes read a 256-byte row of a 32-deep tile); each pair is one
//   16-byte load and its slices 4-byte LDS stores.  (Eight consecutive k per
//   lane instead would touch four times as many cache lines per load.)
// Loads go through a buffer resource whose scalar base walks K, per-lane
// offsets fixed for a segment, so full K tiles cost no vector address
// arithmetic.  Rows outside the problem are clamped to its last row: they
// feed only outputs that are never stored.  In the K tail, offsets at or
// beyond num_records read as zero, and a pair whose second value lies past
// K loads its first value alone.
template <int ROWS, int NT, int BK>
struct Stager {
  static constexpr int KG = BK / 8;       // 8-value groups per row and K tile
  static constexpr int PPR = BK / 2;      // K pairs per row
  static constexpr int LDK = BK + 8;      // LDS row length (bf16)
  static constexpr int NG = ROWS * KG;
  static constexpr int G = (NG + NT - 1) / NT;
  static constexpr bool EXACT = NG % NT == 0;
  static_assert(EXACT || G == 1, "staging shape");
  static_assert(ROWS % 4 == 0 && BK % 8 == 0, "staging shape");
  // An offset past the 2^31 - 1 byte range of every operand, also with any
  // of the scalar offsets added (they stay below 2^31, so the sum does not
  // wrap): its reads return zeros.
  static constexpr uint32_t OOB_K = 0x80000000u;
  const double* base;  // uniform: the block's first row at the current k0
  bool pk;             // uniform: the operand holds packed words
  bool kc;             // uniform: the operand is contiguous in K
  int64_t tstep;       // uniform: elements between K tiles
  uint32_t estep;      // uniform: row-contiguous, bytes between value e and e + 1;
                       // K-contiguous, bytes between pair q and q + 1 (ROWS / 4 rows)
  uint32_t off[G];     // byte offset of value 0 (row-contiguous) or pair 0
  int lds[G];          // LDS index of value 0 or pair 0 in a slice plane
  int nv[G];           // K-contiguous: pairs in rows inside the problem (0..4)

  double v[G][8];

  __device__ __forceinline__ void setup(const double* seg, int ld, bool kc_, int r0, int nrows,
                                        int tid, bool packed) {
    pk = packed;
    kc = kc_;
    base = kc ? seg + (int64_t)r0 * ld : seg + r0;
    tstep = kc ? (int64_t)BK : (int64_t)BK * ld;
    estep = kc ? 8u * (uint32_t)(ROWS / 4) * (uint32_t)ld : 8u * (uint32_t)ld;
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int gi = EXACT ? tid + r * NT : min(tid, NG - 1);
      if (kc) {
        const int kp = gi % PPR, row = gi / PPR;
        const int inside = nrows - r0 - row;  // rows row + q * ROWS / 4 < nrows - r0
        nv[r] = inside <= 0 ? 0 : min(4, (inside + ROWS / 4 - 1) / (ROWS / 4));
        off[r] = (uint32_t)(row * ld + 2 * kp) * 8u;
        lds[r] = row * LDK + 2 * kp;
      } else {
        const int row = gi % ROWS, kg = gi / ROWS;
        const int rc = min(row, nrows - 1 - r0);
        nv[r] = 4;
        off[r] = (uint32_t)(8 * kg * ld + rc) * 8u;
        lds[r] = row * LDK + 8 * kg;
      }
    }
  }

  // Global loads of the K tile starting at k0 (kleft = K - k0 values remain).
  __device__ __forceinline__ void load(int kleft) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, 0x7fffffff, 0x00020000);
    auto pair = [&](int r, int q, uint32_t o) {
      const u4v w = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(rs, o, q * estep, 0));
      v[r][2 * q] = __builtin_bit_cast(double, (uint64_t)w[0] | ((uint64_t)w[1] << 32));
      v[r][2 * q + 1] = __builtin_bit_cast(double, (uint64_t)w[2] | ((uint64_t)w[3] << 32));
    };
    if (kc && kleft >= BK) {
#pragma unroll
      for (int r = 0; r < G; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) pair(r, q, q < nv[r] ? off[r] : OOB_K);
    } else if (kc) {
      // the K tail: each value of a pair loaded on its own, masked by lane
      // (no branch on the lane's K column, which would split the wave)
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int k = lds[r] % LDK;  // the pair's first K column
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool in = q < nv[r];
          v[r][2 * q] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rs, in && k < kleft ? off[r] : OOB_K, q * estep, 0));
          v[r][2 * q + 1] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rs, in && k + 1 < kleft ? off[r] : OOB_K, q * estep + 8, 0));
        }
      }
    } else if (kleft >= BK) {
#pragma unroll
      for (int r = 0; r < G; ++r)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[r][e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off[r], e * estep, 0));
    } else {
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int k0 = lds[r] % LDK;  // the group's first K column
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[r][e] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rs, k0 + e < kleft ? off[r] : OOB_K, e * estep, 0));
      }
    }
  }

  __device__ __forceinline__ void advance() { base += tstep; }

  // The three slice words (values a, b as the low and high halves) of a pair.
  __device__ __forceinline__ void slices(double a, double b, double scale, uint32_t& w0, uint32_t& w1,
                                         uint32_t& w2) const {
    if (pk) {
      const uint64_t u = __builtin_bit_cast(uint64_t, a);
      const uint64_t w = __builtin_bit_cast(uint64_t, b);
      const uint32_t ulo = (uint32_t)u, wlo = (uint32_t)w;
      w0 = (ulo & 0xffffu) | (wlo << 16);
      w1 = (ulo >> 16) | (wlo & 0xffff0000u);
      w2 = (uint32_t)(u >> 32) | ((uint32_t)(w >> 32) << 16);
    } else {
      split_pair(scale * a, scale * b, w0, w1, w2);
    }
  }

  // Split (or unpack) and store into the three slice planes sh[sl][ROWS][LDK];
  // an FP64 operand is multiplied by `scale` first (exact when it is 1).
  __device__ __forceinline__ void store(__bf16 (*sh)[ROWS][LDK], int tid, double scale = 1.0) {
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if (!EXACT && tid >= NG) continue;
      __bf16* p0 = &sh[0][0][0] + lds[r];
      if (kc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t w0, w1, w2;
          slices(v[r][2 * q], v[r][2 * q + 1], scale, w0, w1, w2);
          __bf16* p = p0 + q * (ROWS / 4) * LDK;
          *reinterpret_cast<uint32_t*>(p) = w0;
          *reinterpret_cast<uint32_t*>(p + ROWS * LDK) = w1;
          *reinterpret_cast<uint32_t*>(p + 2 * ROWS * LDK) = w2;
        }
      } else {
        uint32_t w0[4], w1[4], w2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) slices(v[r][2 * q], v[r][2 * q + 1], scale, w0[q], w1[q], w2[q]);
        const u4v s0 = {w0[0], w0[1], w0[2], w0[3]};
        const u4v s1 = {w1[0], w1[1], w1[2], w1[3]};
        const u4v s2 = {w2[0], w2[1], w2[2], w2[3]};
        *reinterpret_cast<u4v*>(p0) = s0;
        *reinterpret_cast<u4v*>(p0 + ROWS * LDK) = s1;
        *reinterpret_cast<u4v*>(p0 + 2 * ROWS * LDK) = s2;
      }
    }
  }
};

template <int BM, int BN, int BK>
constexpr int split_nbuf() {
  return 2 * 3 * (BM + BN) * (BK + 8) * 2 <= 160 * 1024 ? 2 : 1;
}

// NBUF: LDS buffers (0: two where they fit, else one); BK: K tile depth.
// ACC64: FP32 partials flushed into FP64 accumulators (every SPLIT_FLUSH_K
// values and at segment ends, times the segment's alpha); otherwise each
// segment's alpha multiplies its FP64 operand while it is staged and the
// FP32 accumulators hold the whole sum (the plan cuts split-precision sums
// at SPLIT_ACC32_KCHUNK values, so FP32 rounding spans at most that many
// terms before the parts are added in FP64).
template <int BM, int BN, int WGM, int WGN, int NBUF = 0, int BK = SPLIT_BK, bool ACC64 = true>
__device__ __forceinline__ void split_body(Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
                                           const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int NB = NBUF > 0 ? NBUF : split_nbuf<BM, BN, BK>();
  constexpr int LDK = BK + 8;
  constexpr int FLUSH = SPLIT_FLUSH_K / BK > 0 ? SPLIT_FLUSH_K / BK : 1;  // K tiles per FP32 partial
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  static_assert(FM >= 1 && FN >= 1, "tile shape");
  __shared__ __attribute__((aligned(16))) __bf16 Xh[NB][3][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Zh[NB][3][BN][LDK];

  const int64_t lt = xcd_remap_s(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Output sub-tile of this wave, rotated by block so that the waves an edge
  // tile leaves idle fall on different SIMDs from block to block.
  constexpr int NW = WGM * WGN;
  const int role = (wave + 2 * (int)(blockIdx.x & 3)) % NW;
  const int wm = role / WGN, wn = role % WGN;
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  // a wave whose output rows or columns all lie outside the problem issues
  // no fragment reads or MFMAs
  const bool active = m0 + wm * WM < p.M && n0 + wn * WN < p.N;

  f16v acc[FM][FN];
  double acc64[ACC64 ? FM : 1][ACC64 ? FN : 1][ACC64 ? 16 : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[i][j][v] = 0.f;
        if constexpr (ACC64) acc64[i][j][v] = 0.0;
      }
    }

  const int s_end = p.seg0 + p.nseg;
  if (p.nseg > 0) {
    Stager<BM, NT, BK> xs;
    Stager<BN, NT, BK> zs;
    // nk: the K steps of 16 that hold data (the slice planes hold the tile
    // in natural K order, so a segment's last tile skips its zero padding)
    auto mma = [&](int cb, int nk) {
#pragma unroll
      for (int kk = 0; kk < (active ? BK : 0); kk += 16) {
        if (kk >= 16 * nk) break;
        bf8 a[3][FM], b[3][FN];
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
            a[sl][i] = *reinterpret_cast<const bf8*>(&Xh[cb][sl][wm * WM + i * 32 + fr][kk + fk]);
#pragma unroll
          for (int j = 0; j < FN; ++j)
            b[sl][j] = *reinterpret_cast<const bf8*>(&Zh[cb][sl][wn * WN + j * 32 + fr][kk + fk]);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            // smallest products first
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[2][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
          }
      }
    };
    // the FP32 partial sums go into the FP64 ones, times the segment's alpha
    auto flush = [&](double al) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            if constexpr (ACC64) acc64[i][j][v] += al * (double)acc[i][j][v];
            acc[i][j][v] = 0.f;
          }
    };
    // alpha rides on the operator-pool operand (every split segment has
    // one; chosen by buffer, so the pre-split and split-while-staging
    // forms round alike)
    auto pool_z = [](const Seg& q) { return q.zbuf == BUF_LPOOL || q.zbuf == BUF_RPOOL; };
    auto pool_x = [](const Seg& q) { return q.xbuf == BUF_LPOOL || q.xbuf == BUF_RPOOL; };
    // Segments as the outer loop and K tiles as the inner one (the staging
    // layout is fixed in the inner loop, as in the FP64 kernel); inside a
    // segment a tile's global loads go out before the previous tile's MFMAs.
    int s = p.seg0, since_flush = 0, buf = 0;
    Seg g = segs[s];
    xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid, (bases.packed >> g.xbuf) & 1u);
    zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid, (bases.packed >> g.zbuf) & 1u);
    xs.load(g.K);
    zs.load(g.K);
    double sx = 1.0, sz = 1.0;
    if constexpr (!ACC64) (pool_z(g) && !pool_x(g) ? sz : sx) = g.alpha;
    xs.store(Xh[0], tid, sx);
    zs.store(Zh[0], tid, sz);
    __syncthreads();
    while (true) {
      for (int k0 = BK; k0 < g.K; k0 += BK) {
        xs.advance();
        zs.advance();
        xs.load(g.K - k0);
        zs.load(g.K - k0);
        mma(NB == 2 ? buf : 0, BK / 16);
        if (NB == 1) __syncthreads();  // every wave is done with the only buffer
        xs.store(Xh[NB == 2 ? buf ^ 1 : 0], tid, sx);
        zs.store(Zh[NB == 2 ? buf ^ 1 : 0], tid, sz);
        if (ACC64 && ++since_flush == FLUSH) {
          since_flush = 0;
          flush(g.alpha);
        }
        __syncthreads();
        buf ^= 1;
      }
      // the last K tile of segment s; its end flushes the partial sums.  The
      // next segment's layout is derived and its first tile loaded after
      // these MFMAs, so that the layout is not live across them.
      mma(NB == 2 ? buf : 0, g.K > 0 ? (g.K - 1) % BK / 16 + 1 : 0);
      if (++s >= s_end) {
        if constexpr (ACC64) flush(g.alpha);
        break;
      }
      const Seg g2 = segs[s];
      xs.setup(bases.p[g2.xbuf] + g2.xoff, g2.ldx, !g2.xt, m0, p.M, tid, (bases.packed >> g2.xbuf) & 1u);
      zs.setup(bases.p[g2.zbuf] + g2.zoff, g2.ldz, g2.zt, n0, p.N, tid, (bases.packed >> g2.zbuf) & 1u);
      xs.load(g2.K);
      zs.load(g2.K);
      if (NB == 1) __syncthreads();
      sx = 1.0;
      sz = 1.0;
      if constexpr (!ACC64) (pool_z(g2) && !pool_x(g2) ? sz : sx) = g2.alpha;
      xs.store(Xh[NB == 2 ? buf ^ 1 : 0], tid, sx);
      zs.store(Zh[NB == 2 ? buf ^ 1 : 0], tid, sz);
      if constexpr (ACC64) {
        since_flush = 0;
        flush(g.alpha);
      }
      __syncthreads();
      buf ^= 1;
      g = g2;
    }
  }

  double* __restrict__ C = bases.p[p.cbuf] + p.coff;
  if ((bases.packed >> p.cbuf) & 1u) {
    // a packed output (an intermediate; never accumulated): its split words
    uint64_t* __restrict__ Cw = reinterpret_cast<uint64_t*>(C);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          uint32_t s0, s1, s2;
          if constexpr (ACC64)
            split_pair(acc64[i][j][v], acc64[i][j][v + 1], s0, s1, s2);
          else
            split_pair((double)acc[i][j][v], (double)acc[i][j][v + 1], s0, s1, s2);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int m = m0 + wm * WM + i * 32 + 8 * ((v + h) / 4) + 4 * (lane >> 5) + ((v + h) % 4);
            const int n = n0 + wn * WN + j * 32 + fr;
            if (m < p.M && n < p.N) Cw[(int64_t)m * p.ldc + n] = pack_word(s0, s1, s2, h);
          }
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm * WM + i * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int n = n0 + wn * WN + j * 32 + fr;
        if (m < p.M && n < p.N) {
          double* c = C + (int64_t)m * p.ldc + n;
          double r;
          if constexpr (ACC64)
            r = acc64[i][j][v];
          else
            r = (double)acc[i][j][v];
          *c = p.beta ? *c + r : r;
        }
      }
}

template <int BM, int BN, int WGM, int WGN, int NBUF = 0, int BK = SPLIT_BK>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  split_body<BM, BN, WGM, WGN, NBUF, BK, true>(bases, probs, segs, tiles, ntiles);
}

// FP32-accumulating variants: 128 x 128 tiles, two workgroups per CU.
template <int WGM, int WGN, int NBUF, int BK>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(4))) void gemm_split32_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  split_body<128, 128, WGM, WGN, NBUF, BK, false>(bases, probs, segs, tiles, ntiles);
}
dmrg_status launch_gemm_split(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                              const Tile* tiles, hipStream_t s) {
  if (l.ntiles <= 0) return DMRG_OK;
  const Tile* t = tiles + l.tile0;
  dim3 grid((unsigned)l.ntiles);
  switch (l.cfg) {
    case CFG_F64_32:
      gemm_split_kernel<32, 32, 1, 1><<<grid, 64, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64:
      gemm_split_kernel<64, 64, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128:
      gemm_split_kernel<128, 128, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128W8:
      if (split_acc32_variant() > 0)  // eight 32x64 waves, 32-deep K tiles in one 61 KB buffer
        gemm_split32_kernel<4, 2, 1, 32><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      else  // sixteen 32x32 waves, 64-deep K tiles in one LDS buffer, FP64 accumulation
        gemm_split_kernel<128, 128, 4, 4, 1, 64><<<grid, 1024, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64x128:
      gemm_split_kernel<64, 128, 2, 4><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_256x128:
      gemm_split_kernel<256, 128, 4, 4><<<grid, 1024, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

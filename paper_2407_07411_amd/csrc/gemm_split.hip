// Split-precision grouped GEMM: FP64 operands as three BF16 slices on the
// gfx950 BF16 matrix cores, FP32 accumulation over a few K tiles, FP64
// combine.
//
// Each FP64 operand value a is split while it is staged into LDS:
// f = fp32(a), a0 = bf16(f), a1 = bf16(f - a0), a2 = bf16(f - a0 - a1); the
// differences are exact in FP32, so a = a0 + a1 + a2 + O(2^-24 |a|).  The
// product of two split values keeps the six slice products with i + j <= 2
// (the dropped ones are O(2^-24) relative).  Slice products are exact in FP32;
// the matrix cores sum them in FP32, and every SPLIT_FLUSH K tiles the FP32
// partial is added into an FP64 accumulator, which bounds FP32 rounding to
// SPLIT_FLUSH * 32 K values.  Global loads of the next K tile are issued into
// registers before the matrix-core work on the current one.  The
// problem/segment/tile tables and the output-stationary ordering are those of
// the FP64 kernel, so results are deterministic.
//
// Matrix core: v_mfma_f32_32x32x16_bf16.  Lanes: A[i][k] holds i = l%32,
// k = 8(l/32) + e; B[k][j] holds j = l%32, k = 8(l/32) + e (e = 0..7); the 16
// result floats of lane l are D[8(v/4) + 4(l/32) + v%4][l%32] (measured).
#include "internal.h"

namespace dmrg {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int SPLIT_BK = 32;
constexpr int SPLIT_FLUSH = 4;  // K tiles per FP32 partial

__device__ __forceinline__ int64_t xcd_remap_s(int64_t bid, int64_t n) {
  const int64_t per = n / 8, rem = n % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ void split3(double a, __bf16& h0, __bf16& h1, __bf16& h2) {
  const float f = (float)a;
  h0 = (__bf16)f;
  const float r1 = f - (float)h0;
  h1 = (__bf16)r1;
  h2 = (__bf16)(r1 - (float)h1);
}

template <int BM, int BN, int NT>
struct SplitRegs {
  static constexpr int BK = SPLIT_BK;
  static constexpr int NX = (BM * BK + NT - 1) / NT;
  static constexpr int NZ = (BN * BK + NT - 1) / NT;
  double x[NX];
  double z[NZ];

  __device__ __forceinline__ void load(const Seg& g, const double* __restrict__ X,
                                       const double* __restrict__ Z, int k0, int m0, int n0, int M,
                                       int N, int tid) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      const int i = tid + r * NT;
      const int mm = g.xt ? i % BM : i / BK, kk = g.xt ? i / BM : i % BK;
      const int m = m0 + mm, k = k0 + kk;
      const bool ok = i < BM * BK && m < M && k < g.K;
      x[r] = ok ? g.alpha * X[g.xt ? (int64_t)k * g.ldx + m : (int64_t)m * g.ldx + k] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NZ; ++r) {
      const int i = tid + r * NT;
      const int nn = g.zt ? i / BK : i % BN, kk = g.zt ? i % BK : i / BN;
      const int n = n0 + nn, k = k0 + kk;
      const bool ok = i < BN * BK && n < N && k < g.K;
      z[r] = ok ? Z[g.zt ? (int64_t)n * g.ldz + k : (int64_t)k * g.ldz + n] : 0.0;
    }
  }

  template <int LDK>
  __device__ __forceinline__ void store(const Seg& g, __bf16 (*Xh)[BM][LDK], __bf16 (*Zh)[BN][LDK],
                                        int tid) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      const int i = tid + r * NT;
      if (i < BM * BK) {
        const int mm = g.xt ? i % BM : i / BK, kk = g.xt ? i / BM : i % BK;
        split3(x[r], Xh[0][mm][kk], Xh[1][mm][kk], Xh[2][mm][kk]);
      }
    }
#pragma unroll
    for (int r = 0; r < NZ; ++r) {
      const int i = tid + r * NT;
      if (i < BN * BK) {
        const int nn = g.zt ? i / BK : i % BN, kk = g.zt ? i % BK : i / BN;
        split3(z[r], Zh[0][nn][kk], Zh[1][nn][kk], Zh[2][nn][kk]);
      }
    }
  }
};

template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BK = SPLIT_BK, LDK = BK + 8;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  static_assert(FM >= 1 && FN >= 1, "tile shape");
  __shared__ __attribute__((aligned(16))) __bf16 Xh[3][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Zh[3][BN][LDK];

  const int64_t lt = xcd_remap_s(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int fr = lane & 31, fk = (lane >> 5) * 8;

  f16v acc[FM][FN];
  double acc64[FM][FN][16];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[i][j][v] = 0.f;
        acc64[i][j][v] = 0.0;
      }
    }

  const int s_end = p.seg0 + p.nseg;
  if (p.nseg > 0) {
    SplitRegs<BM, BN, NT> regs;
    int s = p.seg0, k0 = 0, since_flush = 0;
    Seg g = segs[s];
    regs.load(g, bases.p[g.xbuf] + g.xoff, bases.p[g.zbuf] + g.zoff, 0, m0, n0, p.M, p.N, tid);
    while (true) {
      regs.template store<LDK>(g, Xh, Zh, tid);
      __syncthreads();
      int s2 = s, k2 = k0 + BK;
      Seg g2 = g;
      if (k2 >= g.K) {
        ++s2;
        k2 = 0;
        if (s2 < s_end) g2 = segs[s2];
      }
      const bool more = s2 < s_end;
      if (more)
        regs.load(g2, bases.p[g2.xbuf] + g2.xoff, bases.p[g2.zbuf] + g2.zoff, k2, m0, n0, p.M, p.N,
                  tid);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        bf8 a[3][FM], b[3][FN];
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
            a[sl][i] = *reinterpret_cast<const bf8*>(&Xh[sl][wm * WM + i * 32 + fr][kk + fk]);
#pragma unroll
          for (int j = 0; j < FN; ++j)
            b[sl][j] = *reinterpret_cast<const bf8*>(&Zh[sl][wn * WN + j * 32 + fr][kk + fk]);
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
      if (++since_flush == SPLIT_FLUSH || !more) {
        since_flush = 0;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              acc64[i][j][v] += (double)acc[i][j][v];
              acc[i][j][v] = 0.f;
            }
      }
      if (!more) break;
      __syncthreads();  // every wave is done with the LDS tile before it is overwritten
      s = s2;
      k0 = k2;
      g = g2;
    }
  }

  double* __restrict__ C = bases.p[p.cbuf] + p.coff;
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
          *c = p.beta ? *c + acc64[i][j][v] : acc64[i][j][v];
        }
      }
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
      gemm_split_kernel<128, 128, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_256x128:
      gemm_split_kernel<256, 128, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

// Split-precision grouped GEMM: FP64 operands as three BF16 slices on the
// gfx950 BF16 matrix cores, FP32 accumulation per K tile, FP64 combine.
//
// Each FP64 operand value a is split on the fly (after the global load, before
// the LDS store) into a = a0 + a1 + a2 + O(2^-24 |a|) with a0 = bf16(a),
// a1 = bf16(a - a0), a2 = bf16(a - a0 - a1); the differences are exact in
// FP64/FP32.  The product of two split values keeps the six slice products
// with i + j <= 2 (the dropped ones are O(2^-24) relative).  Slice products
// are exact in FP32; the MFMA sums them in FP32, and every K tile (32) the
// FP32 partial is added into an FP64 accumulator, which bounds the FP32
// rounding to one tile's worth of terms.  The problem/segment/tile tables and
// the output-stationary ordering are those of the FP64 kernel, so results are
// deterministic.
//
// Matrix core: v_mfma_f32_32x32x16_bf16.  Lanes: A[i][k] holds i = l%32,
// k = 8(l/32) + e; B[k][j] holds j = l%32, k = 8(l/32) + e (e = 0..7); the 16
// result floats of lane l are D[8(v/4) + 4(l/32) + v%4][l%32] (measured).
#include "internal.h"

namespace dmrg {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int64_t xcd_remap_s(int64_t bid, int64_t n) {
  const int64_t per = n / 8, rem = n % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ void split3(double a, __bf16& h0, __bf16& h1, __bf16& h2) {
  h0 = (__bf16)(float)a;
  const float r1 = (float)(a - (double)(float)h0);
  h1 = (__bf16)r1;
  const float r2 = r1 - (float)h1;
  h2 = (__bf16)r2;
}

template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BK = 32, LDK = BK + 8;
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

  for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) {
    const Seg g = segs[s];
    const double* __restrict__ X = bases.p[g.xbuf] + g.xoff;
    const double* __restrict__ Z = bases.p[g.zbuf] + g.zoff;
    const double alpha = g.alpha;
    for (int k0 = 0; k0 < g.K; k0 += BK) {
      if (!g.xt) {
        for (int i = tid; i < BM * BK; i += NT) {
          const int mm = i / BK, kk = i % BK;
          const int m = m0 + mm, k = k0 + kk;
          const double v = (m < p.M && k < g.K) ? alpha * X[(int64_t)m * g.ldx + k] : 0.0;
          split3(v, Xh[0][mm][kk], Xh[1][mm][kk], Xh[2][mm][kk]);
        }
      } else {
        for (int i = tid; i < BM * BK; i += NT) {
          const int mm = i % BM, kk = i / BM;
          const int m = m0 + mm, k = k0 + kk;
          const double v = (m < p.M && k < g.K) ? alpha * X[(int64_t)k * g.ldx + m] : 0.0;
          split3(v, Xh[0][mm][kk], Xh[1][mm][kk], Xh[2][mm][kk]);
        }
      }
      if (!g.zt) {
        for (int i = tid; i < BK * BN; i += NT) {
          const int nn = i % BN, kk = i / BN;
          const int n = n0 + nn, k = k0 + kk;
          const double v = (n < p.N && k < g.K) ? Z[(int64_t)k * g.ldz + n] : 0.0;
          split3(v, Zh[0][nn][kk], Zh[1][nn][kk], Zh[2][nn][kk]);
        }
      } else {
        for (int i = tid; i < BK * BN; i += NT) {
          const int kk = i % BK, nn = i / BK;
          const int n = n0 + nn, k = k0 + kk;
          const double v = (n < p.N && k < g.K) ? Z[(int64_t)n * g.ldz + k] : 0.0;
          split3(v, Zh[0][nn][kk], Zh[1][nn][kk], Zh[2][nn][kk]);
        }
      }
      __syncthreads();
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
      // FP64 combine of this K tile's FP32 partial
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            acc64[i][j][v] += (double)acc[i][j][v];
            acc[i][j][v] = 0.f;
          }
      __syncthreads();
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
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

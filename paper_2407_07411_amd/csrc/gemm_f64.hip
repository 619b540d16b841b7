// Grouped FP64 GEMM on gfx950 matrix cores for the sector contractions of
// the two-site effective Hamiltonian.
//
// Every output tile belongs to one problem C (M x N); a problem is a list of
// K segments C += alpha * X * Z whose operands may be stored transposed.  One
// launch covers thousands of problems of uneven size (the sector GEMMs of all
// operator pairs), so the kernel reads its tile from a table instead of
// deriving it from a regular grid.  Each workgroup owns one output tile and
// walks all of its segments in order, so every sum is computed in a fixed
// order by one workgroup: no atomics, bit-reproducible results.
//
// Pipelining: the (segment, K tile) sequence of a tile is walked as one flat
// stream; after the matrix-core work on the current LDS buffer is issued, the
// global loads of the next K tile go out and land in the other LDS buffer, so
// one barrier separates consecutive K tiles.
//
// Matrix core: v_mfma_f64_16x16x4_f64.  Operand lanes: A[i][k] comes from lane
// i + 16k, B[k][j] from lane j + 16k; the four result doubles of lane l hold
// D[l/16 + 4v][l%16], v = 0..3 (measured on gfx950).
#include <algorithm>

#include "internal.h"
#include "stage.h"
#include "tile_dma.h"

namespace dmrg {

// The 64 x 128 shape is held to 80 VGPRs: six waves per SIMD, which its LDS
// footprint (three workgroups per CU) allows.
template <int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(BM == 64 && BN == 128 ? 6 : 1))) void gemm_f64_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(FM >= 1 && FN >= 1 && BK % 4 == 0, "tile shape");
  __shared__ double Xs[2][BK][BM + 1];
  __shared__ double Zs[2][BK][BN + 1];

  const int64_t lt = xcd_remap(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Output sub-tile of this wave.  Waves are dealt to the four SIMDs in turn
  // (wave w on SIMD w % 4).  For 2 x 4 wave grids the two waves of a SIMD take
  // columns s and s + 2 of different rows, so that an edge tile whose last one
  // or two wave columns (or last wave row) hold no output leaves at most one
  // busy wave per SIMD; the SIMD order rotates by block.  Other grids rotate
  // the row-major order by block.
  constexpr int NW = WGM * WGN;
  int wm, wn;
  if (WGM == 2 && WGN == 4) {
    const int simd = (wave + (int)(blockIdx.x & 3)) & 3, slot = wave >> 2;
    wm = slot;
    wn = slot == 0 ? simd : (simd + 2) & 3;
  } else {
    const int role = (wave + 2 * (int)(blockIdx.x & 3)) % NW;
    wm = role / WGN;
    wn = role % WGN;
  }
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int fr = lane & 15, fk = lane >> 4;
  const bool active = m0 + wm * WM < p.M && n0 + wn * WN < p.N;

  // An accumulating output starts from its old values, loaded here so that
  // their latency overlaps the first K tile (loading them in the epilogue
  // would wait on each one: a store may alias the next load).  Lanes outside
  // the problem read its last row or column and store nothing.
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

  const int s_end = p.seg0 + p.nseg;
  if (p.nseg > 0) {
    Stage<BM, BK, NT> xs;
    Stage<BN, BK, NT> zs;
    // edge tiles: a wave whose output rows or columns all lie outside the
    // problem issues no LDS reads or MFMAs
    // nk: the K steps of 4 that hold data; a segment's last K tile skips the
    // rest (zero padding), the inner loop's full tiles take them all
    auto mma = [&](int b, int nk) {
      if (!active) return;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        if (kk >= 4 * nk) break;
        double a[FM], c[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = Xs[b][kk + fk][wm * WM + i * 16 + fr];
#pragma unroll
        for (int j = 0; j < FN; ++j) c[j] = Zs[b][kk + fk][wn * WN + j * 16 + fr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], c[j], acc[i][j], 0, 0, 0);
      }
    };
    // Loads of the next K tile go out after this tile's MFMAs are issued
    // (measured faster than before them: the matrix-core work of the other
    // waves on the SIMD covers their latency); the other LDS buffer was last
    // read before the previous barrier.  Segments form the outer loop and a
    // segment's K tiles the inner one, so the staging layout stays fixed
    // inside the inner loop and only its scalar base moves: written as one
    // loop over (segment, tile), the compiler carried two copies of the
    // layout and exchanged them through register moves on every tile, and
    // each vector instruction takes issue time from the FP64 MFMAs.
    int s = p.seg0;
    Seg g = segs[s];
    xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
    zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
    xs.load(g.K);
    zs.load(g.K);
    xs.store(&Xs[0][0][0], g.alpha);
    zs.store(&Zs[0][0][0], 1.0);
    __syncthreads();
    int buf = 0;
    while (true) {
      // LDS[buf] holds the first K tile of segment s (a segment with K <= 0
      // stages one tile of zeros and issues no MFMAs)
      for (int k0 = BK; k0 < g.K; k0 += BK) {
        xs.advance();
        zs.advance();
        mma(buf, BK / 4);
        xs.load(g.K - k0);
        zs.load(g.K - k0);
        xs.store(&Xs[buf ^ 1][0][0], g.alpha);
        zs.store(&Zs[buf ^ 1][0][0], 1.0);
        __syncthreads();
        buf ^= 1;
      }
      // LDS[buf] holds the last K tile of segment s; the next segment's
      // layout is derived after its MFMAs, so that it is not live across them
      mma(buf, g.K > 0 ? (g.K - 1) % BK / 4 + 1 : 0);
      if (++s >= s_end) break;
      g = segs[s];
      xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
      zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
      xs.load(g.K);
      zs.load(g.K);
      xs.store(&Xs[buf ^ 1][0][0], g.alpha);
      zs.store(&Zs[buf ^ 1][0][0], 1.0);
      __syncthreads();
      buf ^= 1;
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

// The same grouped GEMM with operands loaded straight into LDS (tile_dma.h).
template <int BM, int BN, int WGM, int WGN, int NST>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(BM == 64 && BN == 128 && NST == 2 ? 6 : 1))) void gemm_f64_dma_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  __shared__ __align__(16) double lds[NST * (BM + BN) * dma::BK];
  const int64_t lt = xcd_remap(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  dma::tile_f64<BM, BN, WGM, WGN, NST>(bases, p, segs, t.tm, t.tn, (int)(blockIdx.x & 3), lds);
}

// FP32-operand form of the same grouped GEMM: operand values are rounded to
// FP32 while they are staged into LDS and multiplied on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32: twice the FP64 rate); the FP32 partial, times the
// segment's alpha, is added into an FP64 accumulator at every segment end and
// every F32_FLUSH_K values of K, which bounds FP32 rounding to that many terms.
// Lanes as for the FP64 MFMA on the operand side; the four result floats of
// lane l are D[4(l/16) + v][l%16] (measured).  Tables, tile order, edge-wave
// skip and load placement are those of the FP64 kernel.
constexpr int F32_FLUSH_K = 128;

template <int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_f32_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int FLUSH = F32_FLUSH_K / BK > 0 ? F32_FLUSH_K / BK : 1;
  static_assert(FM >= 1 && FN >= 1 && BK % 4 == 0, "tile shape");
  __shared__ float Xs[2][BK][BM + 1];
  __shared__ float Zs[2][BK][BN + 1];

  const int64_t lt = xcd_remap(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NW = WGM * WGN;
  int wm, wn;
  if (WGM == 2 && WGN == 4) {
    const int simd = (wave + (int)(blockIdx.x & 3)) & 3, slot = wave >> 2;
    wm = slot;
    wn = slot == 0 ? simd : (simd + 2) & 3;
  } else {
    const int role = (wave + 2 * (int)(blockIdx.x & 3)) % NW;
    wm = role / WGN;
    wn = role % WGN;
  }
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int fr = lane & 15, fk = lane >> 4;
  const bool active = m0 + wm * WM < p.M && n0 + wn * WN < p.N;

  f4 acc[FM][FN];
  double acc64[FM][FN][4];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[i][j][v] = 0.f;
        acc64[i][j][v] = 0.0;
      }

  const int s_end = p.seg0 + p.nseg;
  if (p.nseg > 0) {
    Stage<BM, BK, NT> xs;
    Stage<BN, BK, NT> zs;
    // nk: the K steps of 4 that hold data (as in gemm_f64_kernel)
    auto mma = [&](int b, int nk) {
      if (!active) return;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        if (kk >= 4 * nk) break;
        float a[FM], c[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = Xs[b][kk + fk][wm * WM + i * 16 + fr];
#pragma unroll
        for (int j = 0; j < FN; ++j) c[j] = Zs[b][kk + fk][wn * WN + j * 16 + fr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], c[j], acc[i][j], 0, 0, 0);
      }
    };
    // the FP32 partial sums go into the FP64 ones, times the segment's alpha
    auto flush = [&](double al) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc64[i][j][v] += al * (double)acc[i][j][v];
            acc[i][j][v] = 0.f;
          }
    };
    // segments as the outer loop and K tiles as the inner one, as in
    // gemm_f64_kernel
    int s = p.seg0, since_flush = 0;
    Seg g = segs[s];
    xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
    zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
    xs.load(g.K);
    zs.load(g.K);
    xs.store(&Xs[0][0][0], 1.0);
    zs.store(&Zs[0][0][0], 1.0);
    __syncthreads();
    int buf = 0;
    while (true) {
      for (int k0 = BK; k0 < g.K; k0 += BK) {
        xs.advance();
        zs.advance();
        mma(buf, BK / 4);
        xs.load(g.K - k0);
        zs.load(g.K - k0);
        xs.store(&Xs[buf ^ 1][0][0], 1.0);
        zs.store(&Zs[buf ^ 1][0][0], 1.0);
        if (++since_flush == FLUSH) {
          since_flush = 0;
          flush(g.alpha);
        }
        __syncthreads();
        buf ^= 1;
      }
      // the last K tile of segment s; its end flushes the partial sums
      mma(buf, g.K > 0 ? (g.K - 1) % BK / 4 + 1 : 0);
      since_flush = 0;
      flush(g.alpha);
      if (++s >= s_end) break;
      g = segs[s];
      xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
      zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
      xs.load(g.K);
      zs.load(g.K);
      xs.store(&Xs[buf ^ 1][0][0], 1.0);
      zs.store(&Zs[buf ^ 1][0][0], 1.0);
      __syncthreads();
      buf ^= 1;
    }
  }

  double* __restrict__ C = bases.p[p.cbuf] + p.coff;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * WM + i * 16 + 4 * fk + v;
        const int n = n0 + wn * WN + j * 16 + fr;
        if (m < p.M && n < p.N) {
          double* c = C + (int64_t)m * p.ldc + n;
          *c = p.beta ? *c + acc64[i][j][v] : acc64[i][j][v];
        }
      }
}

dmrg_status launch_gemm_f32(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                            const Tile* tiles, hipStream_t s) {
  const Tile* t = tiles + l.tile0;
  dim3 grid((unsigned)l.ntiles);
  switch (l.cfg) {
    case CFG_F64_32:
      gemm_f32_kernel<32, 32, 32, 1, 1><<<grid, 64, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64:
      gemm_f32_kernel<64, 64, 32, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128:
      gemm_f32_kernel<128, 128, 16, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128W8:
      gemm_f32_kernel<128, 128, 32, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_256x128:
      gemm_f32_kernel<256, 128, 16, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64x128:
      gemm_f32_kernel<64, 128, 32, 2, 4><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

int cfg_bm(int cfg) {
  switch (cfg) {
    case CFG_F64_32: case CFG_D_32x32: return 32;
    case CFG_F64_64: case CFG_F64_64x128: case CFG_D_64x128: case CFG_D_64x128S3: case CFG_D_64x64: return 64;
    case CFG_F64_256x128: return 256;
    default: return 128;
  }
}
int cfg_bn(int cfg) {
  switch (cfg) {
    case CFG_F64_32: case CFG_D_32x32: return 32;
    case CFG_F64_64: case CFG_D_64x64: return 64;
    default: return 128;
  }
}

dmrg_status launch_gemm(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                        const Tile* tiles, hipStream_t s) {
  if (l.ntiles <= 0) return DMRG_OK;
  if (l.split == DMRG_SPLIT_BF16X3) return launch_gemm_split(l, b, probs, segs, tiles, s);
  if (l.split == DMRG_FP32) return launch_gemm_f32(l, b, probs, segs, tiles, s);
  const Tile* t = tiles + l.tile0;
  dim3 grid((unsigned)l.ntiles);
  switch (l.cfg) {
    case CFG_F64_32:
      gemm_f64_kernel<32, 32, 16, 1, 1><<<grid, 64, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64:
      gemm_f64_kernel<64, 64, 16, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128:
      gemm_f64_kernel<128, 128, 16, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_128W8:
      gemm_f64_kernel<128, 128, 16, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_256x128:
      gemm_f64_kernel<256, 128, 16, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_F64_64x128:
      gemm_f64_kernel<64, 128, 16, 2, 4><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_D_64x128:
      gemm_f64_dma_kernel<64, 128, 2, 4, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_D_64x128S3:
      gemm_f64_dma_kernel<64, 128, 2, 4, 3><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_D_128x128:
      gemm_f64_dma_kernel<128, 128, 4, 2, 2><<<grid, 512, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_D_64x64:
      gemm_f64_dma_kernel<64, 64, 2, 2, 2><<<grid, 256, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    case CFG_D_32x32:
      gemm_f64_dma_kernel<32, 32, 1, 1, 2><<<grid, 64, 0, s>>>(b, probs, segs, t, l.ntiles);
      break;
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

// ---------------------------------------------------------------------------
// Diagonal of H_eff: element (i, j) of block B is the sum over the dq = 0
// pairs reaching B of alpha * Adiag[i] * Bdiag[j], summed in list order.
// A workgroup owns 64 x 64 element tiles of one block (thread: one column,
// 16 rows), so each strided diagonal entry it reads serves 64 elements.
constexpr int DIAG_T = 64;
__global__ __launch_bounds__(256) void diag_kernel(const DiagBlock* __restrict__ blocks, int nblocks,
                                                   const DiagItem* __restrict__ items,
                                                   const double* __restrict__ lpool,
                                                   const double* __restrict__ rpool,
                                                   double* __restrict__ out) {
  constexpr int RPT = DIAG_T / 4;  // rows per thread
  const DiagBlock bk = blocks[blockIdx.y];
  const int tx = threadIdx.x % DIAG_T, ty = threadIdx.x / DIAG_T;
  const int tr = (bk.dl + DIAG_T - 1) / DIAG_T, tc = (bk.dr + DIAG_T - 1) / DIAG_T;
  for (int tile = blockIdx.x; tile < tr * tc; tile += gridDim.x) {
    const int i0 = (tile / tc) * DIAG_T, j = (tile % tc) * DIAG_T + tx;
    double acc[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
    for (int it = bk.item0; it < bk.item0 + bk.nitem; ++it) {
      const DiagItem d = items[it];
      const double bb = j < bk.dr ? (d.boff >= 0 ? rpool[d.boff + (int64_t)j * (d.db + 1)] : 1.0) : 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = i0 + ty + 4 * r;
        const double a = i < bk.dl ? (d.aoff >= 0 ? lpool[d.aoff + (int64_t)i * (d.da + 1)] : 1.0) : 0.0;
        acc[r] += d.alpha * a * bb;
      }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = i0 + ty + 4 * r;
      if (i < bk.dl && j < bk.dr) out[bk.off + (int64_t)i * bk.dr + j] = acc[r];
    }
  }
}

dmrg_status launch_diag(const DiagBlock* blocks, int nblocks, const DiagItem* items,
                        const double* lpool, const double* rpool, double* out, int64_t max_elems,
                        hipStream_t s) {
  if (nblocks <= 0) return DMRG_OK;
  int64_t gx = (max_elems + DIAG_T * DIAG_T - 1) / (DIAG_T * DIAG_T);
  if (gx > 256) gx = 256;
  if (gx < 1) gx = 1;
  diag_kernel<<<dim3((unsigned)gx, (unsigned)nblocks), 256, 0, s>>>(blocks, nblocks, items, lpool,
                                                                     rpool, out);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

namespace dmrg {

// C += sum of its partials, in part order (deterministic).  The partials of
// an element are loaded eight at a time and then added in order: one load in
// flight per add (a loop that adds each partial as it arrives) left the
// kernel at a ninth of HBM bandwidth.  A block has fewer than 2^31 elements.
__global__ __launch_bounds__(256) void reduce_kernel(Bases b, const RedBlock* __restrict__ reds, int r0,
                                                     const int64_t* __restrict__ parts) {
  const RedBlock r = reds[r0 + blockIdx.y];
  double* __restrict__ C = b.p[r.cbuf] + r.coff;
  const double* __restrict__ P = b.p[BUF_PART];
  const int64_t* __restrict__ po = parts + r.part0;
  const int n = r.M * r.N;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int i = (int)((unsigned)e / (unsigned)r.N), j = e - i * r.N;
    double* c = C + (int64_t)i * r.ldc + j;
    double acc = *c;
    int k = 0;
    for (; k + 8 <= r.nparts; k += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = P[po[k + u] + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; k < r.nparts; ++k) acc += P[po[k] + e];
    *c = acc;
  }
}

dmrg_status launch_reduce(const Launch& l, const Bases& b, const RedBlock* reds,
                          const int64_t* parts, hipStream_t s) {
  for (int64_t r0 = l.tile0; r0 < l.tile0 + l.ntiles; r0 += 65535) {
    const int64_t n = std::min<int64_t>(65535, l.tile0 + l.ntiles - r0);
    reduce_kernel<<<dim3(32, (unsigned)n), 256, 0, s>>>(b, reds, (int)r0, parts);
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

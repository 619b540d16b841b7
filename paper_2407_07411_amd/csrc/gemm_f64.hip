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
// Matrix core: v_mfma_f64_16x16x4_f64.  Operand lanes: A[i][k] comes from lane
// i + 16k, B[k][j] from lane j + 16k; the four result doubles of lane l hold
// D[l/16 + 4v][l%16], v = 0..3 (measured on gfx950).
#include "internal.h"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));

// blockIdx -> logical tile.  Workgroups are dealt round-robin to the 8 XCDs;
// this remap hands each XCD a contiguous range of the tile table so that
// neighbouring tiles (same problem, shared operand panels) share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n) {
  const int64_t per = n / 8, rem = n % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_f64_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const Tile* __restrict__ tiles, int64_t ntiles) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(FM >= 1 && FN >= 1 && BK % 4 == 0, "tile shape");
  __shared__ double Xs[BK][BM + 1];
  __shared__ double Zs[BK][BN + 1];

  const int64_t lt = xcd_remap(blockIdx.x, ntiles);
  const Tile t = tiles[lt];
  const Prob p = probs[t.prob];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int fr = lane & 15, fk = lane >> 4;

  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) {
    const Seg g = segs[s];
    const double* __restrict__ X = bases.p[g.xbuf] + g.xoff;
    const double* __restrict__ Z = bases.p[g.zbuf] + g.zoff;
    const double alpha = g.alpha;
    for (int k0 = 0; k0 < g.K; k0 += BK) {
      // X tile (BM x BK) -> Xs[k][m]
      if (!g.xt) {
#pragma unroll
        for (int i = tid; i < BM * BK; i += NT) {
          const int mm = i / BK, kk = i % BK;
          const int m = m0 + mm, k = k0 + kk;
          Xs[kk][mm] = (m < p.M && k < g.K) ? alpha * X[(int64_t)m * g.ldx + k] : 0.0;
        }
      } else {
#pragma unroll
        for (int i = tid; i < BM * BK; i += NT) {
          const int mm = i % BM, kk = i / BM;
          const int m = m0 + mm, k = k0 + kk;
          Xs[kk][mm] = (m < p.M && k < g.K) ? alpha * X[(int64_t)k * g.ldx + m] : 0.0;
        }
      }
      // Z tile (BK x BN) -> Zs[k][n]
      if (!g.zt) {
#pragma unroll
        for (int i = tid; i < BK * BN; i += NT) {
          const int nn = i % BN, kk = i / BN;
          const int n = n0 + nn, k = k0 + kk;
          Zs[kk][nn] = (n < p.N && k < g.K) ? Z[(int64_t)k * g.ldz + n] : 0.0;
        }
      } else {
#pragma unroll
        for (int i = tid; i < BK * BN; i += NT) {
          const int kk = i % BK, nn = i / BK;
          const int n = n0 + nn, k = k0 + kk;
          Zs[kk][nn] = (n < p.N && k < g.K) ? Z[(int64_t)n * g.ldz + k] : 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = Xs[kk + fk][wm * WM + i * 16 + fr];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = Zs[kk + fk][wn * WN + j * 16 + fr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
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
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * WM + i * 16 + fk + 4 * v;
        const int n = n0 + wn * WN + j * 16 + fr;
        if (m < p.M && n < p.N) {
          double* c = C + (int64_t)m * p.ldc + n;
          *c = p.beta ? *c + acc[i][j][v] : acc[i][j][v];
        }
      }
}

int cfg_bm(int cfg) { return cfg == CFG_F64_32 ? 32 : cfg == CFG_F64_64 ? 64 : 128; }
int cfg_bn(int cfg) { return cfg_bm(cfg); }

dmrg_status launch_gemm(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                        const Tile* tiles, hipStream_t s) {
  if (l.ntiles <= 0) return DMRG_OK;
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
    default:
      return fail(DMRG_EINVAL, "unknown tile configuration");
  }
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

// ---------------------------------------------------------------------------
// Diagonal of H_eff: element (i, j) of block B is the sum over the dq = 0
// pairs reaching B of alpha * Adiag[i] * Bdiag[j]; blocks are independent, so
// one thread owns one element and sums its pairs in list order.
__global__ void diag_kernel(const DiagBlock* __restrict__ blocks, int nblocks,
                            const DiagItem* __restrict__ items, const double* __restrict__ lpool,
                            const double* __restrict__ rpool, double* __restrict__ out) {
  const DiagBlock bk = blocks[blockIdx.y];
  const int64_t n = (int64_t)bk.dl * bk.dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / bk.dr), j = (int)(e % bk.dr);
    double acc = 0.0;
    for (int it = bk.item0; it < bk.item0 + bk.nitem; ++it) {
      const DiagItem d = items[it];
      const double a = d.aoff >= 0 ? lpool[d.aoff + (int64_t)i * (d.da + 1)] : 1.0;
      const double bb = d.boff >= 0 ? rpool[d.boff + (int64_t)j * (d.db + 1)] : 1.0;
      acc += d.alpha * a * bb;
    }
    out[bk.off + e] = acc;
  }
}

dmrg_status launch_diag(const DiagBlock* blocks, int nblocks, const DiagItem* items,
                        const double* lpool, const double* rpool, double* out, int64_t max_elems,
                        hipStream_t s) {
  if (nblocks <= 0) return DMRG_OK;
  int64_t gx = (max_elems + 255) / 256;
  if (gx > 64) gx = 64;
  if (gx < 1) gx = 1;
  diag_kernel<<<dim3((unsigned)gx, (unsigned)nblocks), 256, 0, s>>>(blocks, nblocks, items, lpool,
                                                                     rpool, out);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

}  // namespace dmrg

// Internal declarations shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmrg_heff.h"

namespace dmrg {

// ---------------------------------------------------------------------------
// Error handling: a thread-local message plus a status code.
void set_error(const std::string& msg);
dmrg_status fail(dmrg_status st, const std::string& msg);
#define DMRG_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::dmrg::fail(DMRG_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Grouped-GEMM work description.  Operands are named by a buffer id and an
// offset so that a plan does not depend on the caller's psi / y pointers; the
// base pointers are passed by value at launch.
enum BufId : uint8_t {
  BUF_PSI = 0,    // input vector of the matvec
  BUF_Y = 1,      // output vector
  BUF_LPOOL = 2,  // left operator pool
  BUF_RPOOL = 3,  // right operator pool
  BUF_WORK = 4,   // intermediates of the two-GEMM chains
  BUF_YBAR = 5,   // upstream gradient (adjoint)
  BUF_GL = 6,     // left pool gradient (adjoint)
  BUF_GR = 7,     // right pool gradient (adjoint)
  BUF_PART = 8,   // partial sums of split long-K problems
  BUF_COUNT = 9
};
struct Bases {
  double* p[BUF_COUNT];
  // Length of each buffer in doubles (bounds the staged loads of the kernels
  // that fetch whole K tiles).
  int64_t len[BUF_COUNT] = {};
  // Bit b set: buffer b holds pre-split operands, one 64-bit word per value
  // with its three BF16 slices in bits 0-15, 16-31 and 32-47 (bits 48-63
  // zero).  Only the split-precision kernel reads or writes such buffers.
  uint32_t packed = 0;
};

// One K segment of an output tile:  C += alpha * X (M x K) * Z (K x N).
//   xt = 0: X[m][k] = x[m*ldx + k]      xt = 1: X[m][k] = x[k*ldx + m]
//   zt = 0: Z[k][n] = z[k*ldz + n]      zt = 1: Z[k][n] = z[n*ldz + k]
struct Seg {
  int64_t xoff, zoff;
  int32_t K, ldx, ldz;
  uint8_t xbuf, zbuf, xt, zt;
  double alpha;
};
static_assert(sizeof(Seg) == 40, "Seg layout");

// One output matrix C (M x N, row stride ldc) = [beta ? C : 0] + sum of its
// segments in order.
struct Prob {
  int64_t coff;
  int32_t M, N, ldc, seg0, nseg;
  uint8_t cbuf, beta, pad0, pad1;
};
static_assert(sizeof(Prob) == 32, "Prob layout");

// One output tile of one problem.
struct Tile {
  int32_t prob;
  int16_t tm, tn;
};
static_assert(sizeof(Tile) == 8, "Tile layout");

// Tile shapes the kernels are instantiated for.
enum TileCfg : int32_t {
  CFG_F64_32 = 0,      // 32x32 tile, 1 wave
  CFG_F64_64 = 1,      // 64x64 tile, 4 waves
  CFG_F64_128 = 2,     // 128x128 tile, 4 waves
  CFG_F64_128W8 = 3,   // 128x128 tile, 8 waves (two per SIMD)
  CFG_F64_256x128 = 4, // 256x128 tile, 8 waves
  CFG_F64_64x128 = 5,  // 64x128 tile, 8 waves of 32x32 (six waves per SIMD fit)
  // FP64 tiles with operands loaded straight into LDS (tile_dma.h)
  CFG_D_64x128 = 6,    // 64x128, 8 waves of 32x32, 2-deep K-tile ring
  CFG_D_64x128S3 = 7,  // 64x128, 8 waves of 32x32, 3-deep ring
  CFG_D_128x128 = 8,   // 128x128, 8 waves of 32x64, 2-deep ring
  CFG_D_64x64 = 9,     // 64x64, 4 waves of 32x32, 2-deep ring
  CFG_D_32x32 = 10,    // 32x32, 1 wave, 2-deep ring
  CFG_F64_COUNT = 11
};
// Shapes the split and FP32-operand kernels are built for.
constexpr int CFG_REDUCED_COUNT = 6;
int cfg_bm(int cfg);
int cfg_bn(int cfg);

// A launch of the grouped GEMM over a contiguous range of the tile table, or
// (cfg == CFG_REDUCE) of the reduction over a range of the RedBlock table.
constexpr int32_t CFG_REDUCE = 100;
struct Launch {
  int32_t cfg;
  int32_t split;     // kernel family: a dmrg_prec value (FP64, split BF16x3, FP32)
  int64_t tile0;
  int64_t ntiles;
  int32_t phase = 0; // launches of one phase are independent of each other
  int32_t ptype = 0; // 0: the phase writes intermediates only, 1: outputs
};

// Long-K problems are cut into K parts that run as separate workgroups: part
// 0 writes the real output, the others write dense partials, and the
// reduction adds the partials to the output in part order (deterministic).
struct RedBlock {
  int64_t coff;    // output offset (in buffer cbuf), dense M x N with row stride ldc
  int32_t M, N, ldc;
  int32_t part0;   // first index into the part-offset table
  int32_t nparts;  // partials to add
  uint8_t cbuf, pad0, pad1, pad2;
};

// K length above which an output problem is cut into parts (a fixed
// constant, so the cut does not depend on the tile shape).
constexpr int64_t KCHUNK = 4096;

// A program: ordered launches over one set of device tables.
struct Program {
  std::vector<Prob> probs;
  std::vector<Seg> segs;
  std::vector<Tile> tiles;
  std::vector<Launch> launches;
  std::vector<RedBlock> reds;
  std::vector<int64_t> red_parts;  // offsets of partials in BUF_PART
  int64_t part_elems = 0;          // BUF_PART doubles needed
  // First problem and first launch of each workspace wave (one entry per
  // wave plus the end), in execution order.
  std::vector<int64_t> wave_prob0, wave_launch0;
  Prob* d_probs = nullptr;
  Seg* d_segs = nullptr;
  Tile* d_tiles = nullptr;
  RedBlock* d_reds = nullptr;
  int64_t* d_red_parts = nullptr;
  dmrg_status upload();
  void release();
  // Host-side bounds proof of every access the kernels will make, given the
  // length (in doubles) of each buffer id.  Run before the first launch.
  dmrg_status validate(const int64_t* buf_len) const;
  // The problem part of that proof for problems [p0, p1) only.
  dmrg_status validate_probs(const int64_t* buf_len, size_t p0, size_t p1) const;
  dmrg_status run(const Bases& b, hipStream_t s, int precision) const;
  // Launches [l0, l1) only (a whole number of phases), in the same form.
  dmrg_status run_range(const Bases& b, hipStream_t s, int precision, size_t l0, size_t l1) const;
  // Two-stream execution (set for the forward program): within a phase the
  // smaller tile shapes run beside the largest one, and a phase's K-split
  // reduction runs beside the next phase when that one writes intermediates
  // only.  Needs a non-null caller stream; otherwise launches run in order.
  bool concurrent = false;
  // When set, run() records prof_ev[2i] / prof_ev[2i + 1] around launch i on
  // the stream that launch goes to (per-launch durations of the real schedule).
  mutable const hipEvent_t* prof_ev = nullptr;
  dmrg_status launch_at(size_t i, const Bases& b, hipStream_t s, int precision) const;
  mutable hipStream_t side[2] = {nullptr, nullptr};
  mutable std::vector<hipEvent_t> events;
  dmrg_status run_concurrent(const Bases& b, hipStream_t s, int precision, size_t l0, size_t l1) const;
  dmrg_status prepare_concurrent();
};

dmrg_status launch_gemm(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                        const Tile* tiles, hipStream_t s);
// Pack n FP64 values into pre-split words (the layout of Bases::packed).
dmrg_status launch_pack_split(const double* x, double* out, int64_t n, hipStream_t s);
dmrg_status launch_gemm_split(const Launch& l, const Bases& b, const Prob* probs, const Seg* segs,
                              const Tile* tiles, hipStream_t s);
// Which FP32-accumulating split kernel serves 128 x 128 tiles (0: none, the
// FP64-accumulating one); its programs cut sums at SPLIT_ACC32_KCHUNK.
int split_acc32_variant();
constexpr int64_t SPLIT_ACC32_KCHUNK = 2048;
dmrg_status launch_reduce(const Launch& l, const Bases& b, const RedBlock* reds,
                          const int64_t* parts, hipStream_t s);

// ---------------------------------------------------------------------------
// Diagonal: per wavefunction block, the dq = 0 pairs that reach it.
struct DiagItem {
  int64_t aoff, boff;   // stored block offsets (-1: identity on that side)
  int32_t da, db;       // stored block sizes (square)
  double alpha;
};
struct DiagBlock {
  int64_t off;
  int32_t dl, dr, item0, nitem;
};
// Looks up the device address of the allocation-free SVD's scratch array on
// `device` (current) once; dmrg_ctx_create calls it.
dmrg_status svd_scratch_init(int device);

dmrg_status launch_diag(const DiagBlock* blocks, int nblocks, const DiagItem* items,
                        const double* lpool, const double* rpool, double* out, int64_t max_elems,
                        hipStream_t s);

}  // namespace dmrg

// ---------------------------------------------------------------------------
// Opaque handle definitions.
struct dmrg_ctx_s {
  int device;
  hipStream_t stream;
};

struct dmrg_basis_s {
  dmrg_ctx_t ctx;
  std::vector<int32_t> qn;   // [n][2]
  std::vector<int64_t> dim;  // [n]
  int find(int32_t n, int32_t sz) const;
};

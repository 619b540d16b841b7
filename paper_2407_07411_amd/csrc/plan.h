// Plan structures of one effective Hamiltonian.
#pragma once

#include <map>
#include <vector>

#include "internal.h"

namespace dmrg {

// One wavefunction block Psi[q_a, Q - q_a].
struct BlockInfo {
  int32_t a, c;      // left / right sector
  int32_t dl, dr;    // rows, columns
  int64_t off;       // offset in psi
};

// One contribution Y[out] += alpha * op(A) X[in] op(B)^T.  A and B name the
// STORED blocks (rows x cols as stored); at / bt say that the stored block
// enters transposed.  kind: 0 two-sided, 1 left only, 2 right only.
struct Item {
  int32_t in, out;
  int64_t aoff;
  int32_t arows, acols;
  int64_t boff;
  int32_t brows, bcols;
  uint8_t at, bt, kind, pad;
  int32_t term;
  double alpha;
};

// Tile configuration per (phase, M bucket, N bucket); -1 = built-in rule.
constexpr int TUNE_BUCKETS = 7;
inline int size_bucket(int x) {
  return x <= 16 ? 0 : x <= 32 ? 1 : x <= 64 ? 2 : x <= 128 ? 3 : x <= 256 ? 4 : x <= 512 ? 5 : 6;
}
struct TuneTable {
  int8_t cfg[2][TUNE_BUCKETS][TUNE_BUCKETS];
  TuneTable() {
    for (auto& a : cfg)
      for (auto& b : a)
        for (auto& c : b) c = -1;
  }
};

struct ProgramBuilder {
  Program prog;
  size_t phase_first = 0;
  int cfg_override = -1;
  int phase_id = 0;                 // 0: intermediates, 1: sums into the outputs
  bool split = false;               // tile rule of the split-precision kernels
  bool reduced = false;             // a split or FP32-operand program (no LDS-load shapes)
  int32_t phase_seq = 0;            // phases closed so far
  const TuneTable* tune = nullptr;
  int32_t add_prob(uint8_t cbuf, int64_t coff, int M, int N, int ldc, bool beta);
  void add_seg(int32_t prob, const Seg& s);
  void close_phase();
};

// One task of the persistent matvec: an output tile (prob >= 0; row tile
// tm, column tile tn & 0x3fff, tile shape tn >> 14) or a chunk of rows of a
// K-cut reduction (prob = -1 - reduction; chunk tm).
struct PTask {
  int32_t prob;
  int16_t tm;
  uint16_t tn;
};
static_assert(sizeof(PTask) == 8, "PTask layout");

// The persistent form of a FP64 forward program: tasks grouped in phases,
// each phase split into eight ranges (persist.hip).
struct Persist {
  bool built = false;
  int nph = 0;
  int grid = 0;
  std::vector<PTask> tasks;
  std::vector<int64_t> qstart;  // [nph * 8 + 1] first task of each (phase, range)
  std::vector<int32_t> ntask;   // [nph] tasks per phase
  PTask* d_tasks = nullptr;
  int64_t* d_qstart = nullptr;
  int32_t* d_ntask = nullptr;
  int32_t* d_ctl = nullptr;     // heads, completions, exit count, give-up flag
  dmrg_status build(const Program& P);
  void release();
  dmrg_status run(const Bases& b, const Program& P, hipStream_t s, int64_t spin_limit) const;
  dmrg_status check(hipStream_t s) const;  // synchronises; reports a give-up
};

// Out-of-core form: the operator pools stay in the caller's pinned host
// memory.  The items are grouped in waves (ranges of the item list); a
// resident wave reads a device copy of its blocks made once at creation, a
// streamed wave reads one of two staging slots that a copy stream fills
// while earlier waves compute (stream.hip).
struct StreamRun {   // one host-to-device copy
  int64_t src, dst, n;  // doubles: offset in the host pool, in the wave's buffer, length
  uint8_t side;         // 0: left pool, 1: right pool
};
struct StreamWave {
  size_t item0, item1;  // item range
  int32_t slot;         // -1: resident copy, else the staging slot
  int64_t run0, nrun;   // copies of a streamed wave
  int64_t len;          // doubles of the buffer the wave reads
};
struct StreamPlan {
  bool on = false;
  std::vector<StreamWave> waves;  // execution order
  std::vector<StreamRun> runs;
  std::vector<int64_t> aoff, boff;  // per item: block offsets in its wave's buffer
  double* cache = nullptr;          // resident blocks, left runs then right runs
  int64_t cache_elems = 0;
  double* slot[2] = {nullptr, nullptr};
  int64_t slot_elems = 0;
  double* diag = nullptr;           // diagonals of the square dq = 0 blocks, compact
  int64_t streamed_elems = 0;       // doubles copied per matvec
  int32_t n_streamed = 0;           // streamed waves
  hipStream_t copy = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
  void release();
};

dmrg_status heff_apply_eager(struct ::dmrg_heff_s* h, const double* psi, double* y);
// SU(2) form (su2.hip): reduced-block layout of total (N, 2S), the items of
// the spin-adapted terms (6j weights folded into the coefficients), and the
// weight itself.
void su2_layout(const dmrg_basis_s* L, const dmrg_basis_s* R, const int32_t Q[2],
                std::vector<BlockInfo>* blocks, int64_t* total);
dmrg_status build_items_su2(struct ::dmrg_heff_s* h, int64_t n_terms, const dmrg_term_su2* terms);
double su2_weight(int tja, int tjc, int tja2, int tjc2, int tk, int tS);
// Workspace doubles of one item's intermediate (0 for one-sided items) and
// its association order (left operator first when cheaper or equal).
int64_t item_need(const struct ::dmrg_heff_s* h, const Item& it, bool* left_first);
// Groups the items into resident and streamed waves for a device budget of
// `device_bytes`, copies the resident blocks and allocates the slots.
dmrg_status build_stream_plan(struct ::dmrg_heff_s* h, int64_t device_bytes);
// Runs the forward program of the current precision wave by wave.
dmrg_status stream_apply(struct ::dmrg_heff_s* h, const Bases& b);
// Diagonal tables of the out-of-core form: square blocks' diagonals gathered
// from the host pools into one compact device array.
dmrg_status stream_diag_tables(struct ::dmrg_heff_s* h, std::vector<DiagItem>& items);
Seg make_seg(uint8_t xbuf, int64_t xoff, int ldx, bool xt, uint8_t zbuf, int64_t zoff, int ldz,
             bool zt, int K, double alpha);
int choose_cfg(int M, int N, bool split);

}  // namespace dmrg

struct dmrg_heff_s {
  dmrg_ctx_t ctx = nullptr;
  std::vector<int32_t> Lqn, Rqn;
  std::vector<int64_t> Ld, Rd;
  int32_t Q[2] = {0, 0};
  std::vector<dmrg::BlockInfo> blocks;
  std::vector<int32_t> blk_of_left;  // left sector -> block or -1 (U(1) form)
  bool su2 = false;                  // spin-adapted form: qn are (N, 2j), Q is (N, 2S)
  int64_t size = 0;
  std::vector<dmrg::Item> items;
  const double* lpool = nullptr;
  const double* rpool = nullptr;
  int64_t llen = 0, rlen = 0;
  double flops = 0.0, bytes = 0.0;
  int prec = DMRG_FP64;
  dmrg::TuneTable tune[3];  // tile shape per (phase, size bucket), per precision
  int64_t work_budget = 0;  // doubles
  double* work = nullptr;
  int64_t work_elems = 0;
  double* psi_pk = nullptr;    // pre-split copy of the input vector (split precision)
  bool split_pack = true;      // split precision stages psi and intermediates pre-split
  double* part = nullptr;      // partials of cut long-K sums (forward)
  int64_t part_elems = 0;      // its length (doubles), the larger of the two programs
  double* adj_part = nullptr;  // the same for the adjoint
  // forward programs, one per precision (tile shapes differ); same waves,
  // workspace offsets and summation order
  dmrg::Program fwdp[3];
  static int prog_index(int p) { return p == DMRG_SPLIT_BF16X3 ? 1 : p == DMRG_FP32 ? 2 : 0; }
  dmrg::Program& fwd() { return fwdp[prog_index(prec)]; }
  dmrg::Program adj;
  bool adj_built = false;
  int adj_mask = 0;
  bool adj_psibar = false, adj_left = false, adj_right = false;
  double* adj_work = nullptr;
  int64_t adj_work_elems = 0;
  // diagonal
  dmrg::DiagBlock* d_dblocks = nullptr;
  dmrg::DiagItem* d_ditems = nullptr;
  int n_dblocks = 0;
  int64_t max_block_elems = 0;
  // out-of-core operators (lpool / rpool are then pinned host memory)
  dmrg::StreamPlan strm;
  // persistent single-launch form of the FP64 forward program
  dmrg::Persist pers;
  int persistent = 0;
  int64_t spin_limit = 2000000000;  // ticks of the 100 MHz counter (20 s)
  // graph cache for the matvec
  int use_graph = 0;
  const double* g_psi = nullptr;
  double* g_y = nullptr;
  int g_prec = -1;
  hipGraphExec_t g_exec = nullptr;
  hipGraph_t g_graph = nullptr;
};

// Host side of the C ABI: contexts, bases, the wavefunction layout and the
// H_eff plan (work lists for the grouped GEMM kernels).
//
// A plan turns the operator-pair terms into "items": one per (term, input
// wavefunction block), plus one per hermitian-conjugate partner.  Each
// two-sided item is a two-GEMM chain Y_out += alpha * op(A) X_in op(B)^T; the
// planner picks the cheaper association (left-first T = op(A) X_in, or
// right-first W = X_in op(B)^T), stores the intermediate in a device
// workspace (phase 1), and sums all intermediates of one output block as one
// long-K GEMM (phase 2).  Items are processed in waves so that the
// intermediates of one wave fit the workspace.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <set>
#include <string>

#include "plan.h"

namespace dmrg {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
dmrg_status fail(dmrg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

dmrg_status Program::upload() {
  release();
  auto put = [](auto& vec, auto** dptr) -> dmrg_status {
    using T = typename std::remove_reference<decltype(vec)>::type::value_type;
    size_t bytes = std::max<size_t>(1, vec.size()) * sizeof(T);
    if (hipMalloc((void**)dptr, bytes) != hipSuccess) {
      *dptr = nullptr;
      return fail(DMRG_ENOMEM, "hipMalloc of plan tables failed");
    }
    if (!vec.empty())
      DMRG_HIP(hipMemcpy(*dptr, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice));
    return DMRG_OK;
  };
  dmrg_status st;
  if ((st = put(probs, &d_probs)) != DMRG_OK) return st;
  if ((st = put(segs, &d_segs)) != DMRG_OK) return st;
  if ((st = put(tiles, &d_tiles)) != DMRG_OK) return st;
  if ((st = put(reds, &d_reds)) != DMRG_OK) return st;
  if ((st = put(red_parts, &d_red_parts)) != DMRG_OK) return st;
  return DMRG_OK;
}

dmrg_status Program::validate_probs(const int64_t* len, size_t p0, size_t p1) const {
  auto in = [&](uint8_t buf, int64_t lo, int64_t hi) {  // [lo, hi] inclusive
    return buf < BUF_COUNT && lo >= 0 && hi < len[buf];
  };
  if (p0 > p1 || p1 > probs.size()) return fail(DMRG_EQN, "plan: problem range outside the table");
  for (size_t pi = p0; pi < p1; ++pi) {
    const Prob& p = probs[pi];
    if (p.M < 1 || p.N < 1 || p.ldc < p.N || p.seg0 < 0 || p.nseg < 0 ||
        (size_t)p.seg0 + p.nseg > segs.size())
      return fail(DMRG_EQN, "plan: malformed problem " + std::to_string(pi));
    if (!in(p.cbuf, p.coff, p.coff + (int64_t)(p.M - 1) * p.ldc + p.N - 1))
      return fail(DMRG_EQN, "plan: output of problem " + std::to_string(pi) + " out of bounds");
    for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) {
      const Seg& g = segs[s];
      if (g.K < 1) return fail(DMRG_EQN, "plan: empty segment");
      const int64_t xhi = g.xt ? g.xoff + (int64_t)(g.K - 1) * g.ldx + p.M - 1
                               : g.xoff + (int64_t)(p.M - 1) * g.ldx + g.K - 1;
      const int64_t zhi = g.zt ? g.zoff + (int64_t)(p.N - 1) * g.ldz + g.K - 1
                               : g.zoff + (int64_t)(g.K - 1) * g.ldz + p.N - 1;
      const bool xok = g.xt ? g.ldx >= p.M : g.ldx >= g.K;
      const bool zok = g.zt ? g.ldz >= g.K : g.ldz >= p.N;
      if (!xok || !zok || !in(g.xbuf, g.xoff, xhi) || !in(g.zbuf, g.zoff, zhi))
        return fail(DMRG_EQN, "plan: operand of problem " + std::to_string(pi) + " out of bounds");
    }
  }
  return DMRG_OK;
}

dmrg_status Program::validate(const int64_t* len) const {
  auto in = [&](uint8_t buf, int64_t lo, int64_t hi) {  // [lo, hi] inclusive
    return buf < BUF_COUNT && lo >= 0 && hi < len[buf];
  };
  if (dmrg_status st = validate_probs(len, 0, probs.size()); st != DMRG_OK) return st;
  for (size_t ri = 0; ri < reds.size(); ++ri) {
    const RedBlock& r = reds[ri];
    if (r.M < 1 || r.N < 1 || r.ldc < r.N || r.part0 < 0 || r.nparts < 1 ||
        (size_t)r.part0 + r.nparts > red_parts.size() ||
        !in(r.cbuf, r.coff, r.coff + (int64_t)(r.M - 1) * r.ldc + r.N - 1))
      return fail(DMRG_EQN, "plan: malformed reduction " + std::to_string(ri));
    for (int k = 0; k < r.nparts; ++k)
      if (!in(BUF_PART, red_parts[r.part0 + k], red_parts[r.part0 + k] + (int64_t)r.M * r.N - 1))
        return fail(DMRG_EQN, "plan: partial of reduction " + std::to_string(ri) + " out of bounds");
  }
  for (const Launch& l : launches) {
    if (l.cfg == CFG_REDUCE) {
      if (l.tile0 < 0 || l.ntiles < 1 || l.tile0 + l.ntiles > (int64_t)reds.size())
        return fail(DMRG_EQN, "plan: reduction launch outside its table");
      continue;
    }
    if (l.tile0 < 0 || l.ntiles < 0 || l.tile0 + l.ntiles > (int64_t)tiles.size())
      return fail(DMRG_EQN, "plan: launch outside the tile table");
    const int bm = cfg_bm(l.cfg), bn = cfg_bn(l.cfg);
    for (int64_t i = l.tile0; i < l.tile0 + l.ntiles; ++i) {
      const Tile& t = tiles[i];
      if (t.prob < 0 || (size_t)t.prob >= probs.size() || t.tm < 0 || t.tn < 0 ||
          (int64_t)t.tm * bm >= probs[t.prob].M || (int64_t)t.tn * bn >= probs[t.prob].N)
        return fail(DMRG_EQN, "plan: tile outside its problem");
    }
  }
  return DMRG_OK;
}

void Program::release() {
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  events.clear();
  for (int i = 0; i < 2; ++i) {
    if (side[i]) (void)hipStreamDestroy(side[i]);
    side[i] = nullptr;
  }
  if (d_probs) (void)hipFree(d_probs);
  if (d_segs) (void)hipFree(d_segs);
  if (d_tiles) (void)hipFree(d_tiles);
  d_probs = nullptr;
  if (d_reds) (void)hipFree(d_reds);
  if (d_red_parts) (void)hipFree(d_red_parts);
  d_segs = nullptr;
  d_tiles = nullptr;
  d_reds = nullptr;
  d_red_parts = nullptr;
}

// Side streams (default priority, non-blocking) and the events of one run,
// created with the plan so that no creation call falls inside a graph capture.
dmrg_status Program::prepare_concurrent() {
  int nphase = 0;
  for (const Launch& l : launches) nphase = std::max(nphase, l.phase + 1);
  for (int i = 0; i < 2; ++i)
    if (!side[i]) DMRG_HIP(hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking));
  const size_t need = 4 * (size_t)nphase + 1;
  while (events.size() < need) {
    hipEvent_t e;
    DMRG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    events.push_back(e);
  }
  concurrent = true;
  return DMRG_OK;
}

dmrg_status Program::run(const Bases& b, hipStream_t s, int precision) const {
  return run_range(b, s, precision, 0, launches.size());
}

dmrg_status Program::launch_at(size_t i, const Bases& b, hipStream_t s, int precision) const {
  Launch x = launches[i];
  x.split = precision;
  if (prof_ev) DMRG_HIP(hipEventRecord(prof_ev[2 * i], s));
  dmrg_status st = x.cfg == CFG_REDUCE ? launch_reduce(x, b, d_reds, d_red_parts, s)
                                       : launch_gemm(x, b, d_probs, d_segs, d_tiles, s);
  if (st == DMRG_OK && prof_ev) DMRG_HIP(hipEventRecord(prof_ev[2 * i + 1], s));
  return st;
}

dmrg_status Program::run_range(const Bases& b, hipStream_t s, int precision, size_t l0, size_t l1) const {
  if (concurrent && s != nullptr) return run_concurrent(b, s, precision, l0, l1);
  for (size_t i = l0; i < l1; ++i)
    if (dmrg_status st = launch_at(i, b, s, precision); st != DMRG_OK) return st;
  return DMRG_OK;
}

// Stream s (the caller's) runs the largest tile shape of every phase; side[0]
// runs the smaller shapes of the same phase (fork after the previous phase,
// join before the next); side[1] runs a K-split reduction next to the
// following phase when that phase writes intermediates only (its outputs and
// the partial sums are not touched there), and the phase after it waits for
// the reduction.  Every side stream is joined into s before returning, so the
// caller sees one ordered operation (and a graph capture on s closes).
dmrg_status Program::run_concurrent(const Bases& b, hipStream_t s, int precision, size_t l0,
                                    size_t l1) const {
  size_t ev = 0;
  hipEvent_t pending = nullptr;  // reduction still running on side[1]
  int pending_phase = -1;
  for (size_t i = l0; i < l1;) {
    const int ph = launches[i].phase;
    size_t j = i;
    while (j < l1 && launches[j].phase == ph) ++j;
    if (pending && ph - pending_phase >= 2) {
      DMRG_HIP(hipStreamWaitEvent(s, pending, 0));
      pending = nullptr;
    }
    std::vector<const Launch*> gemms;
    const Launch* red = nullptr;
    for (size_t k = i; k < j; ++k) {
      if (launches[k].cfg == CFG_REDUCE) red = &launches[k];
      else gemms.push_back(&launches[k]);
    }
    // launches are stored largest tile shape first
    if (gemms.size() > 1) {
      hipEvent_t fork = events[ev++], done = events[ev++];
      DMRG_HIP(hipEventRecord(fork, s));
      DMRG_HIP(hipStreamWaitEvent(side[0], fork, 0));
      for (size_t k = 1; k < gemms.size(); ++k) {
        dmrg_status st = launch_at(gemms[k] - launches.data(), b, side[0], precision);
        if (st != DMRG_OK) return st;
      }
      DMRG_HIP(hipEventRecord(done, side[0]));
      if (!gemms.empty()) {
        dmrg_status st = launch_at(gemms[0] - launches.data(), b, s, precision);
        if (st != DMRG_OK) return st;
      }
      DMRG_HIP(hipStreamWaitEvent(s, done, 0));
    } else if (!gemms.empty()) {
      dmrg_status st = launch_at(gemms[0] - launches.data(), b, s, precision);
      if (st != DMRG_OK) return st;
    }
    if (red) {
      const bool next_intermediate = j < l1 && launches[j].ptype == 0;
      if (next_intermediate) {
        if (pending) {  // at most one reduction in flight
          DMRG_HIP(hipStreamWaitEvent(s, pending, 0));
          pending = nullptr;
        }
        hipEvent_t fork = events[ev++], done = events[ev++];
        DMRG_HIP(hipEventRecord(fork, s));
        DMRG_HIP(hipStreamWaitEvent(side[1], fork, 0));
        dmrg_status st = launch_at(red - launches.data(), b, side[1], precision);
        if (st != DMRG_OK) return st;
        DMRG_HIP(hipEventRecord(done, side[1]));
        pending = done;
        pending_phase = ph;
      } else {
        dmrg_status st = launch_at(red - launches.data(), b, s, precision);
        if (st != DMRG_OK) return st;
      }
    }
    i = j;
  }
  if (pending) DMRG_HIP(hipStreamWaitEvent(s, pending, 0));
  return DMRG_OK;
}

// K length above which output sums are cut (DMRG_HEFF_KCHUNK overrides the
// default, for tests).
int64_t kchunk_from_env() {
  const char* s = std::getenv("DMRG_HEFF_KCHUNK");
  const int64_t v = s ? std::atoll(s) : KCHUNK;
  return v >= 16 ? v : KCHUNK;
}

// Tile shape for one output matrix.  FP64: 64x128 tiles of eight 32x32
// waves (high occupancy, 64-row padding) measured fastest on sector-shaped
// sums; split precision: 128x128 (its three BF16 planes make 64x128 tiles
// LDS-bound at one workgroup per CU).
int choose_cfg(int M, int N, bool split) {
  if (split && M >= 96 && N >= 96) return CFG_F64_128W8;
  if (!split && M >= 40 && N >= 96) return CFG_F64_64x128;
  if (M >= 40 && N >= 40) return CFG_F64_64;
  return CFG_F64_32;
}

// FP64 programs: DMRG_HEFF_DMA selects the LDS-load kernels for the shapes
// above (1: 2-deep ring, 2: 3-deep ring for 64x128, 3: 128x128 for large
// problems); 0 keeps the register-staged kernels.
int dma_mode() {
  const char* s = std::getenv("DMRG_HEFF_DMA");
  return s ? std::atoi(s) : 0;
}
int to_dma(int cfg, int M, int N) {
  const int mode = dma_mode();
  if (mode <= 0) return cfg;
  switch (cfg) {
    case CFG_F64_64x128:
      if (mode == 3 && M >= 96 && N >= 96) return CFG_D_128x128;
      return mode == 2 ? CFG_D_64x128S3 : CFG_D_64x128;
    case CFG_F64_64: return CFG_D_64x64;
    case CFG_F64_32: return CFG_D_32x32;
    default: return cfg;
  }
}

// Appends the tiles of `probs[first..)` grouped by tile configuration, one
// launch per configuration.
void ProgramBuilder::close_phase() {
  // cut long-K problems into parts of about kchunk along segment boundaries
  // split precision with FP32-accumulating tiles: sums cut shorter (the
  // parts are added in FP64 by the ordered reduction)
  const int64_t kchunk = split && split_acc32_variant() > 0 ? std::min(kchunk_from_env(), SPLIT_ACC32_KCHUNK)
                                                           : kchunk_from_env();
  const size_t nprob = prog.probs.size();
  const size_t red_first = prog.reds.size();
  int64_t part_used = 0;
  for (size_t pi = phase_first; pi < nprob; ++pi) {
    Prob p = prog.probs[pi];
    int64_t ktot = 0;
    for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) ktot += prog.segs[s].K;
    if (p.nseg < 2 || ktot <= kchunk) continue;
    const int64_t nparts = std::min<int64_t>((ktot + kchunk - 1) / kchunk, p.nseg);
    const double target = (double)ktot / (double)nparts;
    std::vector<int32_t> cut{p.seg0};
    int64_t acc = 0;
    for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) {
      acc += prog.segs[s].K;
      if (acc >= target * (double)cut.size() && (int64_t)cut.size() < nparts && s + 1 < p.seg0 + p.nseg)
        cut.push_back(s + 1);
    }
    cut.push_back(p.seg0 + p.nseg);
    if (cut.size() <= 2) continue;
    RedBlock r{};
    r.coff = p.coff;
    r.M = p.M;
    r.N = p.N;
    r.ldc = p.ldc;
    r.cbuf = p.cbuf;
    r.part0 = (int32_t)prog.red_parts.size();
    r.nparts = (int32_t)cut.size() - 2;
    prog.probs[pi].nseg = cut[1] - cut[0];
    for (size_t c = 1; c + 1 < cut.size(); ++c) {
      Prob q = p;
      q.cbuf = BUF_PART;
      q.coff = part_used;
      q.ldc = p.N;
      q.beta = 0;
      q.seg0 = cut[c];
      q.nseg = cut[c + 1] - cut[c];
      prog.red_parts.push_back(part_used);
      part_used += (int64_t)p.M * p.N;
      prog.probs.push_back(q);
    }
    prog.reds.push_back(r);
  }
  prog.part_elems = std::max(prog.part_elems, part_used);
  std::vector<std::vector<Tile>> per(CFG_F64_COUNT);
  for (size_t pi = phase_first; pi < prog.probs.size(); ++pi) {
    const Prob& p = prog.probs[pi];
    int cfg = cfg_override;
    if (cfg < 0 && tune) cfg = tune->cfg[phase_id][size_bucket(p.M)][size_bucket(p.N)];
    if (cfg < 0 && (p.cbuf == BUF_GL || p.cbuf == BUF_GR)) {
      // operator-block gradients: one or two short K segments per block;
      // many 32 x 32 tiles beat few padded large ones (adjoint at D=1024:
      // 41.7 -> 25.2 ms against the general rule)
      int64_t kt = 0;
      for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) kt += prog.segs[s].K;
      if (kt <= 512) cfg = CFG_F64_32;
    }
    if (cfg < 0 && !split && p.cbuf != BUF_GL && p.cbuf != BUF_GR && p.M >= 40 && p.N >= 40) {
      // short K sums (<= 256): 64 x 64 tiles (D=1024 forward +4%, D=4096
      // matvec +0.4% against 64 x 128)
      int64_t kt = 0;
      for (int s = p.seg0; s < p.seg0 + p.nseg; ++s) kt += prog.segs[s].K;
      if (kt <= 256) cfg = CFG_F64_64;
    }
    if (cfg < 0) cfg = choose_cfg(p.M, p.N, split);
    if (!split && !reduced && cfg_override < 0) cfg = to_dma(cfg, p.M, p.N);
    prog.probs[pi].pad0 = (uint8_t)phase_id;
    int bm = cfg_bm(cfg), bn = cfg_bn(cfg);
    int tm = (p.M + bm - 1) / bm, tn = (p.N + bn - 1) / bn;
    for (int i = 0; i < tm; ++i)
      for (int j = 0; j < tn; ++j) per[cfg].push_back(Tile{(int32_t)pi, (int16_t)i, (int16_t)j});
  }
  for (int c = CFG_F64_COUNT - 1; c >= 0; --c) {
    if (per[c].empty()) continue;
    Launch l{c, 0, (int64_t)prog.tiles.size(), (int64_t)per[c].size(), phase_seq, phase_id};
    prog.tiles.insert(prog.tiles.end(), per[c].begin(), per[c].end());
    prog.launches.push_back(l);
  }
  if (prog.reds.size() > red_first)
    prog.launches.push_back(Launch{CFG_REDUCE, 0, (int64_t)red_first,
                                   (int64_t)(prog.reds.size() - red_first), phase_seq, phase_id});
  phase_first = prog.probs.size();
  ++phase_seq;
}

int32_t ProgramBuilder::add_prob(uint8_t cbuf, int64_t coff, int M, int N, int ldc, bool beta) {
  Prob p{};
  p.coff = coff;
  p.M = M;
  p.N = N;
  p.ldc = ldc;
  p.seg0 = (int32_t)prog.segs.size();
  p.nseg = 0;
  p.cbuf = cbuf;
  p.beta = beta ? 1 : 0;
  prog.probs.push_back(p);
  return (int32_t)prog.probs.size() - 1;
}

void ProgramBuilder::add_seg(int32_t prob, const Seg& s) {
  // segments of one problem are contiguous: problems are filled one at a time
  prog.segs.push_back(s);
  prog.probs[prob].nseg++;
}

Seg make_seg(uint8_t xbuf, int64_t xoff, int ldx, bool xt, uint8_t zbuf, int64_t zoff, int ldz,
             bool zt, int K, double alpha) {
  Seg s{};
  s.xoff = xoff;
  s.zoff = zoff;
  s.K = K;
  s.ldx = ldx;
  s.ldz = ldz;
  s.xbuf = xbuf;
  s.zbuf = zbuf;
  s.xt = xt ? 1 : 0;
  s.zt = zt ? 1 : 0;
  s.alpha = alpha;
  return s;
}

}  // namespace dmrg

using namespace dmrg;

int dmrg_basis_s::find(int32_t n, int32_t sz) const {
  for (size_t i = 0; i < dim.size(); ++i)
    if (qn[2 * i] == n && qn[2 * i + 1] == sz) return (int)i;
  return -1;
}

extern "C" {

const char* dmrg_last_error(void) { return g_last_error.c_str(); }

const char* dmrg_build_info(void) {
  return "dmrg_heff gfx950: FP64 MFMA 16x16x4 grouped GEMM, BF16x3 split MFMA 32x32x16";
}

dmrg_status dmrg_ctx_create(int device, void* hip_stream, dmrg_ctx_t* out) {
  if (!out) return fail(DMRG_EINVAL, "ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  DMRG_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DMRG_EINVAL, "ctx_create: bad device ordinal");
  DMRG_HIP(hipSetDevice(device));
  if (dmrg_status st = svd_scratch_init(device); st != DMRG_OK) return st;
  auto* c = new (std::nothrow) dmrg_ctx_s{device, (hipStream_t)hip_stream};
  if (!c) return fail(DMRG_ENOMEM, "ctx_create: out of host memory");
  *out = c;
  return DMRG_OK;
}

dmrg_status dmrg_ctx_set_stream(dmrg_ctx_t ctx, void* hip_stream) {
  if (!ctx) return fail(DMRG_EINVAL, "ctx_set_stream: ctx is NULL");
  ctx->stream = (hipStream_t)hip_stream;
  return DMRG_OK;
}

void dmrg_ctx_destroy(dmrg_ctx_t ctx) { delete ctx; }

dmrg_status dmrg_basis_create(dmrg_ctx_t ctx, int32_t n_sec, const int32_t* qn, const int64_t* dim,
                              dmrg_basis_t* out) {
  if (!out) return fail(DMRG_EINVAL, "basis_create: out is NULL");
  *out = nullptr;
  if (!ctx || !qn || !dim || n_sec < 1) return fail(DMRG_EINVAL, "basis_create: bad arguments");
  std::set<std::pair<int32_t, int32_t>> seen;
  for (int i = 0; i < n_sec; ++i) {
    if (dim[i] < 1 || dim[i] > (int64_t)1 << 30)
      return fail(DMRG_EINVAL, "basis_create: sector dimension out of range");
    if (!seen.insert({qn[2 * i], qn[2 * i + 1]}).second)
      return fail(DMRG_EQN, "basis_create: duplicate quantum numbers");
  }
  auto* b = new (std::nothrow) dmrg_basis_s;
  if (!b) return fail(DMRG_ENOMEM, "basis_create: out of host memory");
  b->ctx = ctx;
  b->qn.assign(qn, qn + 2 * n_sec);
  b->dim.assign(dim, dim + n_sec);
  *out = b;
  return DMRG_OK;
}

void dmrg_basis_destroy(dmrg_basis_t b) { delete b; }

dmrg_status dmrg_wfn_layout(dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2], int64_t* n_blocks,
                            int64_t* block_offset, int64_t* total) {
  if (!L || !R || !Q) return fail(DMRG_EINVAL, "wfn_layout: bad arguments");
  int64_t off = 0, nb = 0;
  for (size_t a = 0; a < L->dim.size(); ++a) {
    int c = R->find(Q[0] - L->qn[2 * a], Q[1] - L->qn[2 * a + 1]);
    if (block_offset) block_offset[a] = c < 0 ? -1 : off;
    if (c < 0) continue;
    off += L->dim[a] * R->dim[c];
    ++nb;
  }
  if (n_blocks) *n_blocks = nb;
  if (total) *total = off;
  return DMRG_OK;
}

}  // extern "C"

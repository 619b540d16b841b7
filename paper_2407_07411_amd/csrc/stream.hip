// Out-of-core operators: the operator pools stay in the caller's pinned host
// memory and reach the device in pieces during each matvec.
//
// The paper names host-device traffic as what ends its performance plateau
// once the operators outgrow GPU memory (Performance assessment section:
// bond dimensions beyond about 8000-10000), and hides part of it with
// asynchronous transfers.  Here the items of the forward program (one per
// operator pair and wavefunction block, in term order) are grouped in waves:
//   * a prefix of the items whose distinct blocks fit the resident part of
//     the device budget is copied once, at creation, and its waves read that
//     copy;
//   * the remaining items are cut into waves whose distinct blocks fit one
//     staging slot.  Two slots alternate: a copy stream fills slot k for a
//     streamed wave while the compute stream runs earlier waves, and the
//     compute stream releases the slot when the wave that read it is done.
// Resident and streamed waves are interleaved in proportion (streamed bytes
// against resident FLOPs) so that the copy engine and the matrix cores run
// together; every wave is the same two-phase grouped GEMM as the
// HBM-resident program, reading its operator blocks from the wave's buffer.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "plan.h"

namespace dmrg {

namespace {

// Staging slot size: DMRG_HEFF_STREAM_SLOT_KB, else 1/16 of the device
// budget, at most 1 GiB (doubles; raised to the largest item's blocks by the
// caller).  Small slots leave more of the budget to resident blocks (every
// byte resident is a byte not copied per matvec); 1 GiB of operator blocks
// still holds thousands of output tiles at the paper's bond dimensions.
int64_t slot_doubles(int64_t budget) {
  if (const char* s = std::getenv("DMRG_HEFF_STREAM_SLOT_KB")) {
    const int64_t kb = std::atoll(s);
    if (kb >= 1) return kb * 1024 / 8;
  }
  return std::min<int64_t>(budget / 16, (int64_t)1 << 27);
}

// DMRG_HEFF_STREAM_RESIDENT_KB caps the resident copy below what the budget
// allows (-1: not set); 0 streams every item.
int64_t resident_cap_from_env() {
  const char* s = std::getenv("DMRG_HEFF_STREAM_RESIDENT_KB");
  if (!s) return -1;
  const int64_t kb = std::atoll(s);
  return kb >= 0 ? kb * 1024 / 8 : -1;
}

// Whether [p, p + n) lies in page-locked host memory (hipHostMalloc).
bool pinned_host(const double* p, int64_t n) {
  for (const double* q : {p, p + (n - 1)}) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, q) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (a.type != hipMemoryTypeHost) return false;
  }
  return true;
}

struct Blk {
  uint8_t side;  // 0 left pool, 1 right pool
  int64_t off, n;
  bool operator<(const Blk& o) const {
    return side != o.side ? side < o.side : off != o.off ? off < o.off : n < o.n;
  }
};

int item_blocks(const Item& it, Blk out[2]) {
  int k = 0;
  if (it.aoff >= 0) out[k++] = Blk{0, it.aoff, (int64_t)it.arows * it.acols};
  if (it.boff >= 0) out[k++] = Blk{1, it.boff, (int64_t)it.brows * it.bcols};
  return k;
}

// Lays the distinct blocks of items [i0, i1) out as merged copy runs (left
// runs first), appends the runs, and maps every item's block offsets into
// the resulting buffer.  Returns the buffer length (doubles).
int64_t lay_out(const dmrg_heff_s* h, size_t i0, size_t i1, std::vector<StreamRun>& runs,
                std::vector<int64_t>& aoff, std::vector<int64_t>& boff) {
  std::set<Blk> blks;
  for (size_t i = i0; i < i1; ++i) {
    Blk b[2];
    const int k = item_blocks(h->items[i], b);
    for (int j = 0; j < k; ++j) blks.insert(b[j]);
  }
  const size_t r0 = runs.size();
  int64_t dst = 0;
  for (const Blk& b : blks) {  // sorted by (side, offset): merge overlapping or adjacent blocks
    StreamRun* last = runs.size() > r0 ? &runs.back() : nullptr;
    if (last && last->side == b.side && b.off <= last->src + last->n) {
      const int64_t end = std::max(last->src + last->n, b.off + b.n);
      dst += end - (last->src + last->n);
      last->n = end - last->src;
      continue;
    }
    runs.push_back(StreamRun{b.off, dst, b.n, b.side});
    dst += b.n;
  }
  auto where = [&](uint8_t side, int64_t off) {
    // the run of this side whose source range holds off
    size_t lo = r0, hi = runs.size();
    while (hi - lo > 1) {
      const size_t mid = (lo + hi) / 2;
      const StreamRun& m = runs[mid];
      if (m.side < side || (m.side == side && m.src <= off)) lo = mid;
      else hi = mid;
    }
    const StreamRun& r = runs[lo];
    return r.dst + (off - r.src);
  };
  for (size_t i = i0; i < i1; ++i) {
    const Item& it = h->items[i];
    if (it.aoff >= 0) aoff[i] = where(0, it.aoff);
    if (it.boff >= 0) boff[i] = where(1, it.boff);
  }
  return dst;
}

}  // namespace

void StreamPlan::release() {
  if (copy) (void)hipStreamSynchronize(copy);
  if (cache) (void)hipFree(cache);
  for (double*& p : slot) {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  if (diag) (void)hipFree(diag);
  for (int k = 0; k < 2; ++k) {
    if (copied[k]) (void)hipEventDestroy(copied[k]);
    if (freed[k]) (void)hipEventDestroy(freed[k]);
    copied[k] = freed[k] = nullptr;
  }
  if (copy) (void)hipStreamDestroy(copy);
  cache = nullptr;
  diag = nullptr;
  copy = nullptr;
  on = false;
}

dmrg_status build_stream_plan(dmrg_heff_s* h, int64_t device_bytes) {
  StreamPlan& S = h->strm;
  if (h->llen > 0 && !pinned_host(h->lpool, h->llen))
    return fail(DMRG_EINVAL, "heff_create_streamed: the left pool must be pinned host memory (hipHostMalloc)");
  if (h->rlen > 0 && !pinned_host(h->rpool, h->rlen))
    return fail(DMRG_EINVAL, "heff_create_streamed: the right pool must be pinned host memory (hipHostMalloc)");
  const size_t ni = h->items.size();
  const int64_t budget = device_bytes / 8;
  std::vector<int64_t> need(ni), fp(ni);
  std::vector<double> flops(ni);
  std::set<Blk> all;
  int64_t max_fp = 0;
  for (size_t i = 0; i < ni; ++i) {
    const Item& it = h->items[i];
    bool lf;
    need[i] = item_need(h, it, &lf);
    Blk b[2];
    const int k = item_blocks(it, b);
    fp[i] = 0;
    for (int j = 0; j < k; ++j) {
      fp[i] += b[j].n;
      all.insert(b[j]);
    }
    max_fp = std::max(max_fp, fp[i]);
    const BlockInfo& bi = h->blocks[it.in];
    const BlockInfo& bo = h->blocks[it.out];
    flops[i] = it.kind == 1   ? 2.0 * bo.dl * bi.dl * bi.dr
               : it.kind == 2 ? 2.0 * bi.dl * bi.dr * bo.dr
                              : 2.0 * (double)need[i] * (lf ? bi.dl + bo.dr : bi.dr + bo.dl);
  }
  int64_t distinct = 0;
  for (const Blk& b : all) distinct += b.n;
  // resident prefix: everything when the distinct blocks fit the budget,
  // else the items whose blocks fit beside two staging slots
  const int64_t forced = resident_cap_from_env();
  int64_t slot = 0, cache_cap = budget;
  if (distinct > (forced >= 0 ? std::min(forced, budget) : budget)) {
    slot = std::max(slot_doubles(budget), max_fp);
    if (2 * slot > budget)
      return fail(DMRG_ENOMEM, "heff_create_streamed: a device budget of " + std::to_string(device_bytes) +
                                   " bytes holds less than two staging slots of " +
                                   std::to_string(8 * slot) + " bytes (the largest pair's blocks take " +
                                   std::to_string(8 * max_fp) + ")");
    cache_cap = budget - 2 * slot;
    if (forced >= 0) cache_cap = std::min(cache_cap, forced);
  }
  size_t r = 0;
  {
    std::set<Blk> held;
    int64_t used = 0;
    for (; r < ni; ++r) {
      Blk b[2];
      const int k = item_blocks(h->items[r], b);
      int64_t add = 0;
      for (int j = 0; j < k; ++j)
        if (!held.count(b[j])) add += b[j].n;
      if (used + add > cache_cap) break;
      for (int j = 0; j < k; ++j) held.insert(b[j]);
      used += add;
    }
  }
  const int64_t wb = std::max(h->work_budget, ni ? *std::max_element(need.begin(), need.end()) : 0);
  // waves: streamed ones by workspace and slot; resident ones by workspace
  // and, when there are streamed waves, in about as many pieces of equal
  // FLOPs, so that every streamed wave has resident work to overlap with
  std::vector<StreamWave> res, str;
  {
    size_t w0 = r;
    int64_t used = 0;
    std::set<Blk> held;
    int64_t held_n = 0;
    for (size_t i = r; i < ni; ++i) {
      Blk b[2];
      const int k = item_blocks(h->items[i], b);
      int64_t add = 0;
      for (int j = 0; j < k; ++j)
        if (!held.count(b[j])) add += b[j].n;
      if ((used + need[i] > wb || held_n + add > slot) && i > w0) {
        str.push_back(StreamWave{w0, i, 0, 0, 0, 0});
        w0 = i;
        used = 0;
        held.clear();
        held_n = 0;
        add = fp[i];
      }
      for (int j = 0; j < k; ++j) held.insert(b[j]);
      held_n += add;
      used += need[i];
    }
    if (r < ni) str.push_back(StreamWave{w0, ni, 0, 0, 0, 0});
  }
  {
    double res_flops = 0.0;
    for (size_t i = 0; i < r; ++i) res_flops += flops[i];
    const double piece = str.empty() ? 0.0 : res_flops / (double)str.size();
    size_t w0 = 0;
    int64_t used = 0;
    double acc = 0.0;
    for (size_t i = 0; i < r; ++i) {
      if ((used + need[i] > wb || (piece > 0.0 && acc + 0.5 * flops[i] > piece)) && i > w0) {
        res.push_back(StreamWave{w0, i, -1, 0, 0, 0});
        w0 = i;
        used = 0;
        acc = 0.0;
      }
      used += need[i];
      acc += flops[i];
    }
    if (r > 0 || ni == 0) res.push_back(StreamWave{w0, r, -1, 0, 0, 0});
  }
  // buffers: one resident copy, each streamed wave laid out in its slot
  S.aoff.assign(ni, -1);
  S.boff.assign(ni, -1);
  std::vector<StreamRun> cache_runs;
  S.cache_elems = lay_out(h, 0, r, cache_runs, S.aoff, S.boff);
  S.slot_elems = 0;
  S.streamed_elems = 0;
  for (size_t j = 0; j < str.size(); ++j) {
    StreamWave& W = str[j];
    W.slot = (int32_t)(j & 1);
    W.run0 = (int64_t)S.runs.size();
    W.len = lay_out(h, W.item0, W.item1, S.runs, S.aoff, S.boff);
    W.nrun = (int64_t)S.runs.size() - W.run0;
    S.slot_elems = std::max(S.slot_elems, W.len);
    S.streamed_elems += W.len;
  }
  for (StreamWave& W : res) W.len = S.cache_elems;
  // execution order: merge by the fraction of resident FLOPs and of streamed
  // bytes that precede each wave (resident first on ties, so that the first
  // copy runs beside computation)
  std::vector<double> kr(res.size()), ks(str.size());
  {
    double tot = 0.0, acc = 0.0;
    for (const StreamWave& W : res)
      for (size_t i = W.item0; i < W.item1; ++i) tot += flops[i];
    for (size_t j = 0; j < res.size(); ++j) {
      kr[j] = tot > 0.0 ? acc / tot : 0.0;
      for (size_t i = res[j].item0; i < res[j].item1; ++i) acc += flops[i];
    }
    tot = (double)S.streamed_elems;
    acc = 0.0;
    for (size_t j = 0; j < str.size(); ++j) {
      ks[j] = tot > 0.0 ? acc / tot : 0.0;
      acc += (double)str[j].len;
    }
  }
  S.waves.clear();
  for (size_t a = 0, b = 0; a < res.size() || b < str.size();) {
    if (b == str.size() || (a < res.size() && kr[a] <= ks[b])) S.waves.push_back(res[a++]);
    else S.waves.push_back(str[b++]);
  }
  S.n_streamed = (int32_t)str.size();
  S.on = true;
  // device memory: the resident copy (filled now) and the two slots
  if (S.cache_elems > 0) {
    if (hipMalloc(&S.cache, S.cache_elems * sizeof(double)) != hipSuccess) {
      S.cache = nullptr;
      return fail(DMRG_ENOMEM, "heff_create_streamed: resident operator copy allocation failed");
    }
    for (const StreamRun& R : cache_runs)
      DMRG_HIP(hipMemcpy(S.cache + R.dst, (R.side ? h->rpool : h->lpool) + R.src, R.n * sizeof(double),
                         hipMemcpyHostToDevice));
  }
  if (!str.empty())
    for (int k = 0; k < 2; ++k)
      if (hipMalloc(&S.slot[k], S.slot_elems * sizeof(double)) != hipSuccess) {
        S.slot[k] = nullptr;
        return fail(DMRG_ENOMEM, "heff_create_streamed: staging slot allocation failed");
      }
  DMRG_HIP(hipStreamCreateWithFlags(&S.copy, hipStreamNonBlocking));
  for (int k = 0; k < 2; ++k) {
    DMRG_HIP(hipEventCreateWithFlags(&S.copied[k], hipEventDisableTiming));
    DMRG_HIP(hipEventCreateWithFlags(&S.freed[k], hipEventDisableTiming));
    // both slots start free
    DMRG_HIP(hipEventRecord(S.freed[k], h->ctx->stream));
  }
  return DMRG_OK;
}

dmrg_status stream_apply(dmrg_heff_s* h, const Bases& base) {
  const StreamPlan& S = h->strm;
  const Program& P = h->fwd();
  hipStream_t s = h->ctx->stream, c = S.copy;
  std::vector<size_t> streamed;
  for (size_t w = 0; w < S.waves.size(); ++w)
    if (S.waves[w].slot >= 0) streamed.push_back(w);
  // copies of one streamed wave into its slot, after the slot's last reader
  auto issue = [&](size_t w) -> dmrg_status {
    const StreamWave& W = S.waves[w];
    DMRG_HIP(hipStreamWaitEvent(c, S.freed[W.slot], 0));
    for (int64_t i = W.run0; i < W.run0 + W.nrun; ++i) {
      const StreamRun& R = S.runs[i];
      const double* src = (R.side ? h->rpool : h->lpool) + R.src;
      DMRG_HIP(hipMemcpyAsync(S.slot[W.slot] + R.dst, src, R.n * sizeof(double), hipMemcpyHostToDevice, c));
    }
    DMRG_HIP(hipEventRecord(S.copied[W.slot], c));
    return DMRG_OK;
  };
  size_t next = 0;
  dmrg_status st = DMRG_OK;
  while (st == DMRG_OK && next < streamed.size() && next < 2) st = issue(streamed[next++]);
  for (size_t w = 0; w < S.waves.size() && st == DMRG_OK; ++w) {
    const StreamWave& W = S.waves[w];
    Bases b = base;
    double* buf = W.slot < 0 ? S.cache : S.slot[W.slot];
    b.p[BUF_LPOOL] = b.p[BUF_RPOOL] = buf;
    b.len[BUF_LPOOL] = b.len[BUF_RPOOL] = W.len;
    if (W.slot >= 0) DMRG_HIP(hipStreamWaitEvent(s, S.copied[W.slot], 0));
    st = P.run_range(b, s, h->prec, (size_t)P.wave_launch0[w], (size_t)P.wave_launch0[w + 1]);
    if (st == DMRG_OK && W.slot >= 0) {
      DMRG_HIP(hipEventRecord(S.freed[W.slot], s));
      if (next < streamed.size()) st = issue(streamed[next++]);
    }
  }
  return st;
}

dmrg_status stream_diag_tables(dmrg_heff_s* h, std::vector<DiagItem>& items) {
  StreamPlan& S = h->strm;
  std::map<Blk, int64_t> at;  // (side, block offset, order) -> offset in the compact array
  std::vector<double> vals;
  auto gather = [&](uint8_t side, int64_t off, int32_t d) {
    auto [it, fresh] = at.emplace(Blk{side, off, d}, (int64_t)vals.size());
    if (fresh) {
      const double* p = (side ? h->rpool : h->lpool) + off;
      for (int64_t i = 0; i < d; ++i) vals.push_back(p[i * (d + 1)]);
    }
    return it->second;
  };
  for (DiagItem& di : items) {
    if (di.aoff >= 0) di.aoff = gather(0, di.aoff, di.da);
    if (di.boff >= 0) di.boff = gather(1, di.boff, di.db);
    di.da = di.db = 0;  // unit stride: the diagonal is stored contiguously
  }
  if (hipMalloc(&S.diag, std::max<size_t>(vals.size(), 1) * sizeof(double)) != hipSuccess) {
    S.diag = nullptr;
    return fail(DMRG_ENOMEM, "heff_create_streamed: diagonal table allocation failed");
  }
  if (!vals.empty())
    DMRG_HIP(hipMemcpy(S.diag, vals.data(), vals.size() * sizeof(double), hipMemcpyHostToDevice));
  return DMRG_OK;
}

}  // namespace dmrg

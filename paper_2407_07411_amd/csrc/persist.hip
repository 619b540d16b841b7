// Persistent FP64 matvec: the whole forward program of one H_eff . psi in a
// single launch.
//
// The program's launches are regrouped into phases that must run in order:
// phase q holds the grouped-GEMM problems of program phase q (intermediates
// of one workspace wave, or the long-K output sums that read them) plus the
// K-cut reductions of program phase q - 1 (they touch only the outputs and
// the partial sums, which phase q leaves alone).  Every problem is cut into
// 64 x 128 output tiles; a reduction into chunks of rows.  Each phase's tasks
// are split into eight contiguous ranges, one per XCD (a workgroup serves the
// range of blockIdx % 8 first, then takes what is left in the others), so
// neighbouring tiles of one problem share an L2.
//
// A fixed grid of workgroups (as many as are resident at once) dequeues tasks
// with one atomic counter per (phase, range).  A workgroup takes a task of
// phase p only once every range of every earlier phase has been handed out.
// Before its first task of phase p it publishes how many tasks of its
// previous phase it completed (one atomic add after a device-scope release
// fence) and waits until phase p - 1 is complete (every phase holds at least
// one task, so that implies all earlier phases).  Progress argument: a task
// waits only for tasks of earlier phases; those were all handed out before it
// to workgroups that are running, which finish them without waiting (their
// own waits concern still earlier phases, complete by induction) and publish
// them before they wait for anything themselves.  No workgroup needs to be
// co-resident with another.  Every wait is bounded (spin_limit ticks of the
// 100 MHz real-time counter): past it the workgroup records a give-up flag
// that the host reads (dmrg_heff_check) and carries on, so the grid always
// drains.  The last workgroup to leave resets the counters for the next
// launch, so the kernel needs no clearing step and replays from a hipGraph.
//
// Within a phase a workgroup runs its consecutive GEMM tiles as one stream of
// K tiles: the first K tile of the next tile is loaded while the last K tile
// of the current one is multiplied, and the current tile's results are stored
// while those loads are in flight.  Each element's sum is computed exactly as
// in the per-phase kernels (same segment order, 16-deep K tiles, four K
// values per MFMA step, alpha applied to X before the product, zeros past K,
// reductions adding their parts in order), so the results are bit-identical.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "plan.h"
#include "stage.h"

namespace dmrg {

namespace {

constexpr int P_BM = 64, P_BN = 128, P_BK = 16, P_WGM = 2, P_WGN = 4;  // largest tile shape
constexpr int P_NT = 64 * P_WGM * P_WGN;
constexpr int P_RED_ROWS = 16;

__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(P_NT) __attribute__((amdgpu_waves_per_eu(6))) void persist_f64_kernel(
    Bases bases, const Prob* __restrict__ probs, const Seg* __restrict__ segs,
    const PTask* __restrict__ tasks, const int64_t* __restrict__ qstart,
    const int32_t* __restrict__ phase_tasks, int nph, const RedBlock* __restrict__ reds,
    const int64_t* __restrict__ red_parts, int32_t* __restrict__ ctl, int64_t spin_limit) {
  constexpr int BK = P_BK, NT = P_NT;
  // LDS of the largest tile shape (64 x 128); smaller shapes use a prefix of
  // each buffer with their own row strides
  __shared__ double Xs[2][BK][P_BM + 1];
  __shared__ double Zs[2][BK][P_BN + 1];
  // dequeued task and its phase; two slots so that a slot is rewritten only
  // after every thread has read it (a barrier lies between)
  __shared__ int64_t sh_task[2];
  __shared__ int32_t sh_phase[2], sh_last;

  int32_t* head = ctl;            // [nph * 8] next index per (phase, range)
  int32_t* done = ctl + nph * 8;  // [nph] completed tasks per phase
  int32_t* exitc = done + nph;    // workgroups that have left
  int32_t* flag = exitc + 1;      // set when a wait gave up

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int xq = blockIdx.x & 7;
  // wave roles as in the per-phase kernel, rotated by workgroup
  const int simd = (wave + (int)((blockIdx.x >> 3) & 3)) & 3, slot = wave >> 2;
  const int wm = slot, wn = slot == 0 ? simd : (simd + 2) & 3;

  // Thread 0: the next task at or after phase `from` (-1 when none is left),
  // into shared slot `sl`.
  auto dequeue = [&](int from, int sl) {
    int64_t t = -1;
    int p = from;
    for (; p < nph; ++p) {
      for (int i = 0; i < 8 && t < 0; ++i) {
        const int q = p * 8 + ((xq + i) & 7);
        const int64_t n = qstart[q + 1] - qstart[q];
        if (n <= 0 || ld_relaxed(head + q) >= n) continue;
        const int32_t k = __hip_atomic_fetch_add(head + q, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k < n) t = qstart[q] + k;
      }
      if (t >= 0) break;
    }
    sh_task[sl] = t;
    sh_phase[sl] = p;
  };

  int ph = 0;        // phase of the tasks completed since the last publication
  int32_t mine = 0;  // their number

  // Publish this workgroup's completions of phase ph (all threads).
  auto publish = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0 && mine > 0) __hip_atomic_fetch_add(done + ph, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mine = 0;
  };
  // Wait until every task of phase p - 1 is complete (all threads).
  auto wait_phase = [&](int p) {
    if (tid == 0 && p > 0) {
      const int32_t need = phase_tasks[p - 1];
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (ld_relaxed(done + p - 1) < need) {
        __builtin_amdgcn_s_sleep(4);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > spin_limit) {
          __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  };

  if (tid == 0) dequeue(0, 0);
  __syncthreads();
  int64_t cur = sh_task[0];
  int cph = sh_phase[0];
  __syncthreads();

  while (cur >= 0) {
    if (cph != ph) {
      publish();
      ph = cph;
      wait_phase(ph);
    }
    const PTask T = tasks[cur];
    if (T.prob < 0) {
      // ---- reduction chunk: C += its partial sums, in part order
      const RedBlock r = reds[-T.prob - 1];
      double* __restrict__ C = bases.p[r.cbuf] + r.coff;
      const double* __restrict__ Pp = bases.p[BUF_PART];
      const int r0 = T.tm * P_RED_ROWS, r1 = min(r.M, r0 + P_RED_ROWS);
      for (int64_t e = (int64_t)r0 * r.N + tid; e < (int64_t)r1 * r.N; e += NT) {
        const int64_t i = e / r.N, j = e % r.N;
        double acc = C[i * r.ldc + j];
        for (int k = 0; k < r.nparts; ++k) acc += Pp[red_parts[r.part0 + k] + e];
        C[i * r.ldc + j] = acc;
      }
      ++mine;
      __syncthreads();
      if (tid == 0) dequeue(ph, 0);
      __syncthreads();
      cur = sh_task[0];
      cph = sh_phase[0];
      __syncthreads();
      continue;
    }

    // ---- a chain of GEMM tiles of this phase and tile shape, one stream of
    // K tiles.  The loads run one K tile ahead of the matrix-core work; the
    // tile whose loads are issued and the tile being summed switch together,
    // in the iteration whose loads fetch the next tile's first K tile.
    auto chain = [&](auto bm_c, auto bn_c) {
      constexpr int BM = decltype(bm_c)::value, BN = decltype(bn_c)::value;
      constexpr int WM = BM / P_WGM, WN = BN / P_WGN, FM = WM / 16, FN = WN / 16;
      constexpr int XLD = BM + 1, ZLD = BN + 1;  // LDS row strides (K-major tiles)
      double* const Xb = &Xs[0][0][0];
      double* const Zb = &Zs[0][0][0];
      const int mode = T.tn >> 14;
      // The lane index is passed through an empty asm statement wherever the
      // row and column offsets of the output are derived (start and end of
      // each tile), so that they are recomputed there instead of being held
      // in registers across the K loop.
      auto lane_fr_fk = [&](int* fr_, int* fk_) {
        int tl = tid;
        asm volatile("" : "+v"(tl));
        *fr_ = tl & 15;
        *fk_ = (tl & 63) >> 4;
      };
      int fr, fk;
      lane_fr_fk(&fr, &fk);
      Prob p = probs[T.prob];
      int m0 = T.tm * BM, n0 = (T.tn & 0x3fff) * BN;
      bool act = m0 + wm * WM < p.M && n0 + wn * WN < p.N;
      d4 acc[FM][FN];
      // An accumulating output starts from its old values (buffer loads:
      // out-of-range offsets read as zero when beta = 0, so no branch).
      // Element offsets within one output block fit 32 bits.
      auto init_acc = [&]() {
        int fr, fk;
        lane_fr_fk(&fr, &fk);
        const __amdgpu_buffer_rsrc_t rs = operand_rsrc(bases.p[p.cbuf] + p.coff);
        const bool beta = p.beta != 0;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int m = min(m0 + wm * WM + i * 16 + fk + 4 * v, p.M - 1);
              const int n = min(n0 + wn * WN + j * 16 + fr, p.N - 1);
              const uint32_t off = beta ? (uint32_t)(m * p.ldc + n) * 8u : OOB;
              acc[i][j][v] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
            }
      };
      auto store_acc = [&]() {
        int fr, fk;
        lane_fr_fk(&fr, &fk);
        char* __restrict__ C = (char*)(bases.p[p.cbuf] + p.coff);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int m = m0 + wm * WM + i * 16 + fk + 4 * v;
              const int n = n0 + wn * WN + j * 16 + fr;
              if (m < p.M && n < p.N) *(double*)(C + (uint32_t)(m * p.ldc + n) * 8u) = acc[i][j][v];
            }
      };
      init_acc();
      __syncthreads();  // the LDS buffers may still be read by the previous chain
      if (p.nseg == 0) {  // a block nothing reaches: written as zeros
        store_acc();
        ++mine;
        if (tid == 0) dequeue(ph, 0);
        __syncthreads();
        cur = sh_task[0];
        cph = sh_phase[0];
        __syncthreads();
        return;
      }
      Stage<BM, BK, NT> xs;
      Stage<BN, BK, NT> zs;
      // nk: the K steps of 4 that hold data (a segment's last K tile skips
      // its zero padding, as in the per-phase kernel)
      auto mma = [&](int b, int nk) {
        if (!act) return;
        const double* X = Xb + b * BK * XLD;
        const double* Z = Zb + b * BK * ZLD;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          if (kk >= 4 * nk) break;
          double a[FM], c[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) a[i] = X[(kk + fk) * XLD + wm * WM + i * 16 + fr];
#pragma unroll
          for (int j = 0; j < FN; ++j) c[j] = Z[(kk + fk) * ZLD + wn * WN + j * 16 + fr];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], c[j], acc[i][j], 0, 0, 0);
        }
      };
      int s = p.seg0;
      Seg g = segs[s];
      xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
      zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
      xs.load(g.K);
      zs.load(g.K);
      xs.store(Xb, g.alpha);
      zs.store(Zb, 1.0);
      if (tid == 0) dequeue(ph, 0);  // the task after this one, fetched ahead
      __syncthreads();
      int64_t nxt = sh_task[0];
      int nxph = sh_phase[0];
      int nd = 1;  // dequeues of this chain (slot of the next one: nd & 1)
      int buf = 0;
      // Segments as the outer loop and K tiles as the inner one, as in the
      // per-phase kernel; past the end of this tile's sum the chain moves on
      // to the next task when that is a GEMM tile of this phase and shape with
      // something to sum.
      while (true) {
        for (int k0 = BK; k0 < g.K; k0 += BK) {
          xs.advance();
          zs.advance();
          mma(buf, BK / 4);
          xs.load(g.K - k0);
          zs.load(g.K - k0);
          xs.store(Xb + (buf ^ 1) * BK * XLD, g.alpha);
          zs.store(Zb + (buf ^ 1) * BK * ZLD, 1.0);
          __syncthreads();
          buf ^= 1;
        }
        // the last K tile of segment s
        mma(buf, g.K > 0 ? (g.K - 1) % BK / 4 + 1 : 0);
        if (++s < p.seg0 + p.nseg) {
          g = segs[s];
          xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, m0, p.M, tid);
          zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, n0, p.N, tid);
          xs.load(g.K);
          zs.load(g.K);
          xs.store(Xb + (buf ^ 1) * BK * XLD, g.alpha);
          zs.store(Zb + (buf ^ 1) * BK * ZLD, 1.0);
          __syncthreads();
          buf ^= 1;
          continue;
        }
        int32_t nprob = -1;
        if (nxt >= 0 && nxph == ph) {
          const PTask U = tasks[nxt];
          if (U.prob >= 0 && (U.tn >> 14) == mode && probs[U.prob].nseg > 0) nprob = U.prob;
        }
        if (nprob < 0) break;
        const PTask U = tasks[nxt];
        const Prob q = probs[nprob];
        const int nm0 = U.tm * BM, nn0 = (U.tn & 0x3fff) * BN;
        s = q.seg0;
        g = segs[s];
        xs.setup(bases.p[g.xbuf] + g.xoff, g.ldx, !g.xt, nm0, q.M, tid);
        zs.setup(bases.p[g.zbuf] + g.zoff, g.ldz, g.zt, nn0, q.N, tid);
        xs.load(g.K);
        zs.load(g.K);
        if (tid == 0) dequeue(ph, nd & 1);  // the task after the next, read after the barrier
        xs.store(Xb + (buf ^ 1) * BK * XLD, g.alpha);
        zs.store(Zb + (buf ^ 1) * BK * ZLD, 1.0);
        // this tile's sum is complete: store it, start the next one
        store_acc();
        ++mine;
        p = q;
        m0 = nm0;
        n0 = nn0;
        act = m0 + wm * WM < p.M && n0 + wn * WN < p.N;
        init_acc();
        __syncthreads();
        nxt = sh_task[nd & 1];
        nxph = sh_phase[nd & 1];
        ++nd;
        buf ^= 1;
      }
      store_acc();
      ++mine;
      cur = nxt;
      cph = nxph;
      __syncthreads();  // the shared slots may be rewritten by the next dequeue
    };
    chain(std::integral_constant<int, P_BM>(), std::integral_constant<int, P_BN>());
  }

  // leave: publish, and the last workgroup out resets the counters
  publish();
  if (tid == 0) {
    const int32_t e = __hip_atomic_fetch_add(exitc, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh_last = e == (int32_t)gridDim.x - 1;
  }
  __syncthreads();
  if (sh_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int i = tid; i < nph * 9 + 1; i += NT) ctl[i] = 0;  // heads, done, exit count
  }
}

}  // namespace

// Phases of the persistent form of a forward program (see the file comment).
dmrg_status Persist::build(const Program& P) {
  release();
  const int nprog = P.launches.empty() ? 0 : P.launches.back().phase + 1;
  std::vector<std::vector<PTask>> ph(nprog + 1);
  std::vector<std::vector<double>> work(nprog + 1);
  std::vector<uint8_t> seen(P.probs.size(), 0);
  for (const Launch& l : P.launches) {
    if (l.cfg == CFG_REDUCE) {
      for (int64_t r = l.tile0; r < l.tile0 + l.ntiles; ++r) {
        const RedBlock& rb = P.reds[r];
        for (int c = 0; c * P_RED_ROWS < rb.M; ++c) {
          ph[l.phase + 1].push_back(PTask{(int32_t)(-1 - r), (int16_t)c, (uint16_t)0});
          const int rows = std::min(P_RED_ROWS, rb.M - c * P_RED_ROWS);
          work[l.phase + 1].push_back(8.0 * rows * rb.N * (rb.nparts + 2));  // ~ a byte counts as a FLOP
        }
      }
      continue;
    }
    for (int64_t t = l.tile0; t < l.tile0 + l.ntiles; ++t) {
      const int32_t pi = P.tiles[t].prob;
      if (seen[pi]) continue;
      seen[pi] = 1;
      const Prob& p = P.probs[pi];
      int64_t ktot = 0;
      for (int sg = p.seg0; sg < p.seg0 + p.nseg; ++sg) ktot += P.segs[sg].K;
      // every problem in 64 x 128 tiles (measured: 64 x 64 and 32 x 64 tiles
      // on eight waves for the narrow problems made the D=4096 matvec 21%
      // slower, their registers being shared with the main path)
      const int mode = 0;
      const int bm = P_BM, bn = P_BN;
      const int tm = (p.M + bm - 1) / bm, tn = (p.N + bn - 1) / bn;
      if (tm > 32767 || tn > 0x3fff) return fail(DMRG_ENOTSUP, "persistent matvec: problem too large");
      for (int i = 0; i < tm; ++i)
        for (int j = 0; j < tn; ++j) {
          ph[l.phase].push_back(PTask{pi, (int16_t)i, (uint16_t)(j | (mode << 14))});
          work[l.phase].push_back(2.0 * bm * bn * std::max<int64_t>(ktot, 16));
        }
    }
  }
  // drop empty phases; reductions of a phase lead the next one (they gate
  // the phase after it)
  tasks.clear();
  qstart.clear();
  ntask.clear();
  for (size_t q = 0; q < ph.size(); ++q) {
    if (ph[q].empty()) continue;
    std::vector<size_t> order(ph[q].size());
    size_t o = 0;
    for (size_t i = 0; i < ph[q].size(); ++i)
      if (ph[q][i].prob < 0) order[o++] = i;
    for (size_t i = 0; i < ph[q].size(); ++i)
      if (ph[q][i].prob >= 0) order[o++] = i;
    double total = 0.0;
    for (double w : work[q]) total += w;
    const int64_t base = (int64_t)tasks.size();
    double acc = 0.0;
    int cut = 1;
    qstart.push_back(base);
    for (size_t k = 0; k < order.size(); ++k) {
      tasks.push_back(ph[q][order[k]]);
      acc += work[q][order[k]];
      while (cut < 8 && acc >= total * cut / 8.0) {
        qstart.push_back((int64_t)tasks.size());
        ++cut;
      }
    }
    while (cut < 8) {
      qstart.push_back((int64_t)tasks.size());
      ++cut;
    }
    ntask.push_back((int32_t)(tasks.size() - base));
  }
  qstart.push_back((int64_t)tasks.size());
  nph = (int)ntask.size();
  if ((int64_t)tasks.size() > INT32_MAX) return fail(DMRG_ENOTSUP, "persistent matvec: too many tasks");
  // bounds of every task (the programs' own tables are validated separately)
  for (const PTask& t : tasks) {
    if (t.prob >= 0) {
      const Prob& p = P.probs[t.prob];
      const int mode = t.tn >> 14, tn = t.tn & 0x3fff;
      if (mode != 0 || t.tm < 0 || (int64_t)t.tm * P_BM >= p.M || (int64_t)tn * P_BN >= p.N)
        return fail(DMRG_EQN, "persistent matvec: tile outside its problem");
    } else {
      const int64_t r = -1 - (int64_t)t.prob;
      if (r >= (int64_t)P.reds.size() || t.tm < 0 || (int64_t)t.tm * P_RED_ROWS >= P.reds[r].M)
        return fail(DMRG_EQN, "persistent matvec: reduction chunk outside its block");
    }
  }
  auto put = [](const auto& vec, auto** dptr) -> dmrg_status {
    using T = typename std::decay<decltype(vec)>::type::value_type;
    const size_t bytes = std::max<size_t>(1, vec.size()) * sizeof(T);
    if (hipMalloc((void**)dptr, bytes) != hipSuccess) {
      *dptr = nullptr;
      return fail(DMRG_ENOMEM, "persistent matvec: table allocation failed");
    }
    if (!vec.empty()) DMRG_HIP(hipMemcpy(*dptr, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice));
    return DMRG_OK;
  };
  dmrg_status st;
  if ((st = put(tasks, &d_tasks)) != DMRG_OK || (st = put(qstart, &d_qstart)) != DMRG_OK ||
      (st = put(ntask, &d_ntask)) != DMRG_OK) {
    release();
    return st;
  }
  const size_t nctl = (size_t)nph * 9 + 2;
  if (hipMalloc(&d_ctl, nctl * sizeof(int32_t)) != hipSuccess) {
    d_ctl = nullptr;
    release();
    return fail(DMRG_ENOMEM, "persistent matvec: counter allocation failed");
  }
  DMRG_HIP(hipMemset(d_ctl, 0, nctl * sizeof(int32_t)));
  int dev = 0, cus = 0, per = 0;
  DMRG_HIP(hipGetDevice(&dev));
  DMRG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  DMRG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persist_f64_kernel, P_NT, 0));
  grid = std::max(8, std::min<int>(cus * std::max(per, 1), (int)std::max<size_t>(tasks.size(), 8)));
  built = true;
  return DMRG_OK;
}

void Persist::release() {
  if (d_tasks) (void)hipFree(d_tasks);
  if (d_qstart) (void)hipFree(d_qstart);
  if (d_ntask) (void)hipFree(d_ntask);
  if (d_ctl) (void)hipFree(d_ctl);
  d_tasks = nullptr;
  d_qstart = nullptr;
  d_ntask = nullptr;
  d_ctl = nullptr;
  built = false;
}

dmrg_status Persist::run(const Bases& b, const Program& P, hipStream_t s, int64_t spin_limit) const {
  if (!built) return fail(DMRG_EINVAL, "persistent matvec: schedule not built");
  if (nph == 0) return DMRG_OK;
  persist_f64_kernel<<<grid, P_NT, 0, s>>>(b, P.d_probs, P.d_segs, d_tasks, d_qstart, d_ntask, nph, P.d_reds,
                                           P.d_red_parts, d_ctl, spin_limit);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

dmrg_status Persist::check(hipStream_t s) const {
  if (!built) return DMRG_OK;
  int32_t f = 0;
  DMRG_HIP(hipMemcpyAsync(&f, d_ctl + (size_t)nph * 9 + 1, sizeof(f), hipMemcpyDeviceToHost, s));
  DMRG_HIP(hipStreamSynchronize(s));
  if (f) {
    const int32_t zero = 0;
    DMRG_HIP(hipMemcpyAsync(d_ctl + (size_t)nph * 9 + 1, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return fail(DMRG_EHIP, "persistent matvec: a wait for an earlier phase gave up (results not valid)");
  }
  return DMRG_OK;
}

}  // namespace dmrg

// Davidson eigensolver for the lowest eigenpair of H_eff, run on the device.
//
// The paper's DMRG spends most of its time in the Lanczos/Davidson solve of
// each update (Numerical procedure section); this is E. R. Davidson's method
// (J. Comput. Phys. 17, 87 (1975)) with the diagonal preconditioner,
// two-pass classical Gram-Schmidt and thick restart from the lowest Ritz
// vectors.  All vector work is FP64 and stays on the device; the subspace
// size k lives in device memory so that one iteration is a fixed sequence of
// launches that can be captured once in a hipGraph and replayed:
//
//   stage A: Jacobi eigensolve of the k x k projected matrix G (one
//            workgroup), Ritz vector x = V s, residual r = W s - theta x and
//            ||r|| (deterministic two-level reductions), status to the host;
//   stage B: restart when k is at the maximum, preconditioner, two passes of
//            Gram-Schmidt, normalisation, the matvec w = H t, and the update
//            of V, W, G and k.
//
// The first step runs stage A alone; every later step is ONE launch
// sequence (one graph) of stage B followed by the next stage A, so an
// iteration costs one graph launch and one host synchronisation: the host
// reads the small status record at the end and stops when the residual
// reaches the tolerance.  When stage B's correction vanishes (the stall
// flag), the update of V, W, G and k and the whole of the following stage A
// skip on the device, so the state, the Ritz pair and the residual stay
// those of the last complete iteration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "plan.h"

namespace dmrg {

constexpr int KMAX = 32;         // largest subspace
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 512;  // first-level reduction blocks

struct DavState {
  int32_t k;          // current subspace size
  int32_t stalled;    // correction vanished after orthogonalisation
  double theta;       // lowest Ritz value
  double res;         // ||H x - theta x||
  double evals[KMAX];
};

// ---------------------------------------------------------------------------
// Block-level sum of KR values per thread; results land in red[0..KR).
template <int KR>
__device__ void block_sum(double (&v)[KR], double* red /* [KR][RED_THREADS] */) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < KR; ++i) red[i * RED_THREADS + tid] = v[i];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s)
#pragma unroll
      for (int i = 0; i < KR; ++i) red[i * RED_THREADS + tid] += red[i * RED_THREADS + tid + s];
    __syncthreads();
  }
}

// partial[b][i] = sum over block b's elements of rows[i][e] * vec[e], i < nrows.
// nrows = *kp + kadd (read on the device).
__global__ __launch_bounds__(RED_THREADS) void multidot_kernel(const double* __restrict__ rows,
                                                               const double* __restrict__ vec,
                                                               int64_t n, const DavState* st,
                                                               int kadd, double* __restrict__ partial) {
  __shared__ double red[4 * RED_THREADS];
  const int nrows = min(st->k + kadd, KMAX);
  for (int i0 = 0; i0 < nrows; i0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * RED_THREADS) {
      const double x = vec[e];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + j < nrows) acc[j] += rows[(int64_t)(i0 + j) * n + e] * x;
    }
    block_sum<4>(acc, red);
    if (threadIdx.x < 4 && i0 + threadIdx.x < nrows)
      partial[(int64_t)blockIdx.x * KMAX + i0 + threadIdx.x] = red[threadIdx.x * RED_THREADS];
    __syncthreads();
  }
}

// out[i] = sum_b partial[b][i] in fixed order, i < nrows.
__global__ __launch_bounds__(RED_THREADS) void finish_dot_kernel(const double* __restrict__ partial,
                                                                 int nblocks, const DavState* st,
                                                                 int kadd, double* __restrict__ out) {
  __shared__ double red[RED_THREADS];
  const int nrows = min(st->k + kadd, KMAX);
  for (int i = 0; i < nrows; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) acc += partial[(int64_t)b * KMAX + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

// Jacobi eigensolver of the symmetric k x k matrix G (row stride KMAX), one
// workgroup.  Parallel cyclic ordering: each round rotates k/2 disjoint
// (p, q) pairs chosen by the round-robin tournament, A <- J^T A J, E <- E J.
// Rotation from the standard formulas: theta = (a_qq - a_pp) / (2 a_pq),
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1/sqrt(t^2+1), s = t c.
// Output: eigenvalues ascending in st->evals, eigenvectors as columns of E
// (row stride KMAX) in the same order, st->theta = lowest.
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ G, DavState* st,
                                                     double* __restrict__ Eout) {
  if (st->stalled) return;  // the last correction vanished: keep the last Ritz pair
  __shared__ double A[KMAX][KMAX + 1];
  __shared__ double E[KMAX][KMAX + 1];
  __shared__ double cs[KMAX / 2][2];
  __shared__ int pr[KMAX / 2][2];
  __shared__ int order[KMAX];
  __shared__ double offn, totn;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int k = st->k;
  for (int e = tid; e < KMAX * KMAX; e += nt) {
    const int i = e / KMAX, j = e % KMAX;
    A[i][j] = (i < k && j < k) ? 0.5 * (G[i * KMAX + j] + G[j * KMAX + i]) : 0.0;
    E[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m = k + (k & 1);  // even number of players; player k (if any) is a bye
  for (int sweep = 0; sweep < 40 && k > 1; ++sweep) {
    if (tid == 0) {
      double o = 0.0, t = 0.0;
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          const double a2 = A[i][j] * A[i][j];
          t += a2;
          if (i != j) o += a2;
        }
      offn = o;
      totn = t;
    }
    __syncthreads();
    if (!(offn > 1e-32 * totn) || offn == 0.0) break;
    for (int r = 0; r < m - 1; ++r) {
      if (tid < m / 2) {
        // round-robin: player 0 fixed, players 1..m-1 rotate by r
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (m - 1); };
        int p = player(tid), q = player(m - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < k && A[p][q] != 0.0) {
          const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        pr[tid][0] = p;
        pr[tid][1] = q < k ? q : p;
        cs[tid][0] = c;
        cs[tid][1] = q < k ? s : 0.0;
      }
      __syncthreads();
      // columns: A <- A J, E <- E J
      for (int e = tid; e < (m / 2) * k; e += nt) {
        const int pi = e / k, row = e % k;
        const int p = pr[pi][0], q = pr[pi][1];
        if (p == q) continue;
        const double c = cs[pi][0], s = cs[pi][1];
        const double ap = A[row][p], aq = A[row][q];
        A[row][p] = c * ap - s * aq;
        A[row][q] = s * ap + c * aq;
        const double ep = E[row][p], eq = E[row][q];
        E[row][p] = c * ep - s * eq;
        E[row][q] = s * ep + c * eq;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < (m / 2) * k; e += nt) {
        const int pi = e / k, col = e % k;
        const int p = pr[pi][0], q = pr[pi][1];
        if (p == q) continue;
        const double c = cs[pi][0], s = cs[pi][1];
        const double ap = A[p][col], aq = A[q][col];
        A[p][col] = c * ap - s * aq;
        A[q][col] = s * ap + c * aq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    for (int i = 0; i < k; ++i) order[i] = i;
    for (int i = 1; i < k; ++i) {  // insertion sort, ascending eigenvalue
      int v = order[i], j = i - 1;
      while (j >= 0 && A[order[j]][order[j]] > A[v][v]) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = v;
    }
    for (int i = 0; i < k; ++i) st->evals[i] = A[order[i]][order[i]];
    st->theta = A[order[0]][order[0]];
  }
  __syncthreads();
  for (int e = tid; e < KMAX * KMAX; e += nt) {
    const int i = e / KMAX, j = e % KMAX;
    Eout[i * KMAX + j] = (i < k && j < k) ? E[i][order[j]] : 0.0;
  }
}

// x = V s, hx = W s (s = first eigenvector), r = hx - theta x; partial ||r||^2.
__global__ __launch_bounds__(RED_THREADS) void ritz_kernel(const double* __restrict__ V,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ E,
                                                           const DavState* st, int64_t n,
                                                           double* __restrict__ x, double* __restrict__ r,
                                                           double* __restrict__ partial) {
  if (st->stalled) return;
  __shared__ double red[RED_THREADS];
  __shared__ double s[KMAX];
  const int k = st->k;
  if (threadIdx.x < KMAX) s[threadIdx.x] = threadIdx.x < k ? E[threadIdx.x * KMAX] : 0.0;
  __syncthreads();
  const double theta = st->theta;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (int64_t)gridDim.x * RED_THREADS) {
    double xv = 0.0, hv = 0.0;
    for (int i = 0; i < k; ++i) {
      xv += s[i] * V[(int64_t)i * n + e];
      hv += s[i] * W[(int64_t)i * n + e];
    }
    const double rv = hv - theta * xv;
    x[e] = xv;
    r[e] = rv;
    acc += rv * rv;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int t = RED_THREADS / 2; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * KMAX] = red[0];
}

__global__ void finish_res_kernel(const double* __restrict__ partial, int nblocks, DavState* st) {
  if (st->stalled) return;
  __shared__ double red[RED_THREADS];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) acc += partial[(int64_t)b * KMAX];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) st->res = sqrt(red[0]);
}

// Restart (only when k == kmax): R[j] = sum_i B[i] E[i][j], j < keep.
__global__ void restart_combine_kernel(const double* __restrict__ B, const double* __restrict__ E,
                                       const DavState* st, int kmax, int keep, int64_t n,
                                       double* __restrict__ R) {
  if (st->k != kmax) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    for (int j = 0; j < keep; ++j) {
      double acc = 0.0;
      for (int i = 0; i < kmax; ++i) acc += E[i * KMAX + j] * B[(int64_t)i * n + e];
      R[(int64_t)j * n + e] = acc;
    }
}

__global__ void restart_copy_kernel(const double* __restrict__ R, const DavState* st, int kmax,
                                    int64_t count, double* __restrict__ B) {
  if (st->k != kmax) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    B[e] = R[e];
}

__global__ void restart_finish_kernel(DavState* st, int kmax, int keep, double* __restrict__ G) {
  if (st->k != kmax) return;
  for (int e = threadIdx.x; e < KMAX * KMAX; e += blockDim.x) {
    const int i = e / KMAX, j = e % KMAX;
    G[e] = (i == j && i < keep) ? st->evals[i] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) st->k = keep;
}

// t = r / (theta - d) with |theta - d| clamped to >= 1e-8 (sign kept).
__global__ void precond_kernel(const double* __restrict__ r, const double* __restrict__ d,
                               const DavState* st, int64_t n, double* __restrict__ t) {
  const double theta = st->theta;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double den = theta - d[e];
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    t[e] = r[e] / den;
  }
}

// t -= sum_{i<k} c[i] V[i]
__global__ void subtract_kernel(const double* __restrict__ V, const double* __restrict__ c,
                                const DavState* st, int64_t n, double* __restrict__ t) {
  __shared__ double cc[KMAX];
  const int k = st->k;
  if (threadIdx.x < KMAX) cc[threadIdx.x] = threadIdx.x < k ? c[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = t[e];
    for (int i = 0; i < k; ++i) acc -= cc[i] * V[(int64_t)i * n + e];
    t[e] = acc;
  }
}

// t /= ||t|| (norm^2 in dots[0]); a norm below `floor` flags a vanished
// correction.
__global__ void normalize_kernel(const double* __restrict__ dots, DavState* st, int64_t n,
                                 double* __restrict__ t, double floor) {
  const double nrm = sqrt(dots[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->stalled = !(nrm >= floor);
  if (!(nrm >= floor)) return;
  const double inv = 1.0 / nrm;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    t[e] *= inv;
}

// V[k] = t, W[k] = w
__global__ void append_kernel(const double* __restrict__ t, const double* __restrict__ w,
                              const DavState* st, int64_t n, double* __restrict__ V, double* __restrict__ W) {
  if (st->stalled) return;  // a vanished correction is not added to the subspace
  const int k = st->k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    V[(int64_t)k * n + e] = t[e];
    W[(int64_t)k * n + e] = w[e];
  }
}

// G[i][k] = G[k][i] = dots[i], i <= k; k += 1.
__global__ void grow_kernel(const double* __restrict__ dots, DavState* st, double* __restrict__ G) {
  if (st->stalled) return;
  const int k = st->k;
  for (int i = threadIdx.x; i <= k; i += blockDim.x) {
    G[i * KMAX + k] = dots[i];
    G[k * KMAX + i] = dots[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) st->k = k + 1;
}

__global__ void set_state_kernel(DavState* st, int k) {
  st->k = k;
  st->stalled = 0;
  st->theta = 0.0;
  st->res = 0.0;
}

__global__ void copy_kernel(const double* __restrict__ a, int64_t n, double* __restrict__ b) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

// b -= a
__global__ void diff_kernel(const double* __restrict__ a, int64_t n, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] -= a[i];
}

__global__ void zero_kernel(double* __restrict__ b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = 0.0;
}

// (value, index) of the smallest entry, lowest index on ties: per block into
// partial[b*KMAX + {0,1}], then one block over the partials sets t = e_argmin.
__device__ __forceinline__ bool less_vi(double v, double i, double w, double j) {
  return v < w || (v == w && i < j);
}

__global__ __launch_bounds__(RED_THREADS) void argmin_partial_kernel(const double* __restrict__ d,
                                                                     int64_t n, double* __restrict__ partial) {
  __shared__ double rv[RED_THREADS], ri[RED_THREADS];
  double bv = INFINITY, bi = 1e300;
  for (int64_t e = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (int64_t)gridDim.x * RED_THREADS)
    if (less_vi(d[e], (double)e, bv, bi)) {
      bv = d[e];
      bi = (double)e;
    }
  rv[threadIdx.x] = bv;
  ri[threadIdx.x] = bi;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && less_vi(rv[threadIdx.x + s], ri[threadIdx.x + s], rv[threadIdx.x], ri[threadIdx.x])) {
      rv[threadIdx.x] = rv[threadIdx.x + s];
      ri[threadIdx.x] = ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[(int64_t)blockIdx.x * KMAX] = rv[0];
    partial[(int64_t)blockIdx.x * KMAX + 1] = ri[0];
  }
}

__global__ __launch_bounds__(RED_THREADS) void argmin_finish_kernel(const double* __restrict__ partial,
                                                                    int nblocks, int64_t n,
                                                                    double* __restrict__ t) {
  __shared__ double rv[RED_THREADS], ri[RED_THREADS];
  double bv = INFINITY, bi = 1e300;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
    if (less_vi(partial[(int64_t)b * KMAX], partial[(int64_t)b * KMAX + 1], bv, bi)) {
      bv = partial[(int64_t)b * KMAX];
      bi = partial[(int64_t)b * KMAX + 1];
    }
  rv[threadIdx.x] = bv;
  ri[threadIdx.x] = bi;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && less_vi(rv[threadIdx.x + s], ri[threadIdx.x + s], rv[threadIdx.x], ri[threadIdx.x])) {
      rv[threadIdx.x] = rv[threadIdx.x + s];
      ri[threadIdx.x] = ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t i = ri[0] < (double)n ? (int64_t)ri[0] : 0;  // all-NaN diagonal: first element
    t[i] = 1.0;
  }
}

// partial[b * KMAX] = sum over block b's elements of a[e] * b[e]
__global__ __launch_bounds__(RED_THREADS) void scalar_dot_kernel(const double* __restrict__ a,
                                                                 const double* __restrict__ b, int64_t n,
                                                                 double* __restrict__ partial) {
  __shared__ double red[RED_THREADS];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (int64_t)gridDim.x * RED_THREADS)
    acc += a[e] * b[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int t = RED_THREADS / 2; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * KMAX] = red[0];
}

__global__ void finish_scalar_kernel(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  __shared__ double red[RED_THREADS];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) acc += partial[(int64_t)b * KMAX];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace dmrg

using namespace dmrg;

struct dmrg_dav_s {
  dmrg_heff_t h = nullptr;
  dmrg_dav_opts o{};
  int64_t n = 0;
  double* mem = nullptr;  // one allocation for every vector
  double *V, *W, *RV, *RW, *t, *w, *x, *r, *diag, *G, *E, *partial, *dots;
  DavState* st = nullptr;
  DavState* host = nullptr;  // pinned
  int iters = 0, matvecs = 0, tail = 0;
  bool done = false;
  bool started = false;  // stage A of the first step has run
  hipGraphExec_t gA = nullptr, gB = nullptr;  // gB: stage B + stage A
  hipGraph_t grA = nullptr, grB = nullptr;
};

namespace {

unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

// dots[0..k+kadd) = rows^T vec
dmrg_status multidot(dmrg_dav_s* d, const double* rows, const double* vec, int kadd, hipStream_t s) {
  multidot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(rows, vec, d->n, d->st, kadd, d->partial);
  finish_dot_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, d->st, kadd, d->dots);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

dmrg_status stage_a(dmrg_dav_s* d, hipStream_t s) {
  jacobi_kernel<<<1, 256, 0, s>>>(d->G, d->st, d->E);
  ritz_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d->V, d->W, d->E, d->st, d->n, d->x, d->r, d->partial);
  finish_res_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, d->st);
  DMRG_HIP(hipGetLastError());
  DMRG_HIP(hipMemcpyAsync(d->host, d->st, sizeof(DavState), hipMemcpyDeviceToHost, s));
  return DMRG_OK;
}

// matvec of t into w, then V[k] = t, W[k] = w, G column, k += 1
dmrg_status expand(dmrg_dav_s* d, hipStream_t s) {
  dmrg_status st = heff_apply_eager(d->h, d->t, d->w);
  if (st != DMRG_OK) return st;
  const unsigned g = grid_for(d->n);
  append_kernel<<<g, 256, 0, s>>>(d->t, d->w, d->st, d->n, d->V, d->W);
  DMRG_HIP(hipGetLastError());
  if ((st = multidot(d, d->V, d->w, 1, s)) != DMRG_OK) return st;
  grow_kernel<<<1, 64, 0, s>>>(d->dots, d->st, d->G);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

dmrg_status stage_b(dmrg_dav_s* d, hipStream_t s) {
  const int kmax = d->o.max_subspace, keep = d->o.restart_keep;
  const unsigned g = grid_for(d->n);
  restart_combine_kernel<<<g, 256, 0, s>>>(d->V, d->E, d->st, kmax, keep, d->n, d->RV);
  restart_combine_kernel<<<g, 256, 0, s>>>(d->W, d->E, d->st, kmax, keep, d->n, d->RW);
  restart_copy_kernel<<<g, 256, 0, s>>>(d->RV, d->st, kmax, (int64_t)keep * d->n, d->V);
  restart_copy_kernel<<<g, 256, 0, s>>>(d->RW, d->st, kmax, (int64_t)keep * d->n, d->W);
  restart_finish_kernel<<<1, 256, 0, s>>>(d->st, kmax, keep, d->G);
  precond_kernel<<<g, 256, 0, s>>>(d->r, d->diag, d->st, d->n, d->t);
  // unit correction first, so that the test after orthogonalisation is
  // relative: it stalls only when t lies in the subspace to ~1e-12
  scalar_dot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d->t, d->t, d->n, d->partial);
  finish_scalar_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, d->dots);
  normalize_kernel<<<g, 256, 0, s>>>(d->dots, d->st, d->n, d->t, 1e-300);
  DMRG_HIP(hipGetLastError());
  for (int pass = 0; pass < 2; ++pass) {
    dmrg_status st = multidot(d, d->V, d->t, 0, s);
    if (st != DMRG_OK) return st;
    subtract_kernel<<<g, 256, 0, s>>>(d->V, d->dots, d->st, d->n, d->t);
    DMRG_HIP(hipGetLastError());
  }
  scalar_dot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d->t, d->t, d->n, d->partial);
  finish_scalar_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, d->dots);
  normalize_kernel<<<g, 256, 0, s>>>(d->dots, d->st, d->n, d->t, 1e-12);
  DMRG_HIP(hipGetLastError());
  return expand(d, s);
}

// One iteration after the first: the correction and matvec, then the next
// Ritz pair and the status record for the host.
dmrg_status stage_ba(dmrg_dav_s* d, hipStream_t s) {
  dmrg_status st = stage_b(d, s);
  return st == DMRG_OK ? stage_a(d, s) : st;
}

void free_dav(dmrg_dav_s* d) {
  if (!d) return;
  if (d->gA) (void)hipGraphExecDestroy(d->gA);
  if (d->gB) (void)hipGraphExecDestroy(d->gB);
  if (d->grA) (void)hipGraphDestroy(d->grA);
  if (d->grB) (void)hipGraphDestroy(d->grB);
  if (d->mem) (void)hipFree(d->mem);
  if (d->st) (void)hipFree(d->st);
  if (d->host) (void)hipHostFree(d->host);
  delete d;
}

template <class F>
dmrg_status run_stage(dmrg_dav_s* d, hipGraphExec_t* exec, hipGraph_t* graph, F&& body) {
  hipStream_t s = d->h->ctx->stream;
  if (!d->o.use_graph) return body(d, s);
  if (!*exec) {
    if (s == nullptr) return fail(DMRG_EINVAL, "davidson: graph capture needs a non-null stream");
    DMRG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    dmrg_status st = body(d, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != DMRG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(DMRG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    *graph = g;
    DMRG_HIP(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  }
  DMRG_HIP(hipGraphLaunch(*exec, s));
  return DMRG_OK;
}

}  // namespace

extern "C" {

dmrg_status dmrg_davidson_create(dmrg_heff_t h, const dmrg_dav_opts* opts, const double* psi0,
                                 dmrg_dav_t* out) {
  if (!out) return fail(DMRG_EINVAL, "davidson_create: out is NULL");
  *out = nullptr;
  if (!h || !opts || (!psi0 && opts->start != 1) || opts->start < 0 || opts->start > 1)
    return fail(DMRG_EINVAL, "davidson_create: bad arguments");
  const dmrg_dav_opts& o = *opts;
  if (o.max_subspace < 2 || o.max_subspace > KMAX || o.restart_keep < 1 ||
      o.restart_keep >= o.max_subspace || o.max_iter < 0 || !(o.tol >= 0.0) || o.fp64_tail < 0)
    return fail(DMRG_EINVAL, "davidson_create: bad options (2 <= max_subspace <= 32, "
                             "1 <= restart_keep < max_subspace, tol >= 0)");
  std::unique_ptr<dmrg_dav_s, void (*)(dmrg_dav_s*)> d(new (std::nothrow) dmrg_dav_s, free_dav);
  if (!d) return fail(DMRG_ENOMEM, "davidson_create: out of host memory");
  d->h = h;
  d->o = o;
  // out-of-core operators: the matvec's copies and cross-stream waits stay
  // eager, so the stages run without graphs
  if (h->strm.on) d->o.use_graph = 0;
  const int64_t n = h->size;
  d->n = n;
  const int kmax = o.max_subspace, keep = o.restart_keep;
  const int64_t vec_doubles = (int64_t)(2 * kmax + 2 * keep + 5) * n;
  const int64_t small = (int64_t)2 * KMAX * KMAX + (int64_t)RED_BLOCKS * KMAX + KMAX;
  if (hipMalloc(&d->mem, (vec_doubles + small) * sizeof(double)) != hipSuccess) {
    d->mem = nullptr;
    return fail(DMRG_ENOMEM, "davidson_create: device allocation failed");
  }
  double* p = d->mem;
  d->V = p; p += (int64_t)kmax * n;
  d->W = p; p += (int64_t)kmax * n;
  d->RV = p; p += (int64_t)keep * n;
  d->RW = p; p += (int64_t)keep * n;
  d->t = p; p += n;
  d->w = p; p += n;
  d->x = p; p += n;
  d->r = p; p += n;
  d->diag = p; p += n;
  d->G = p; p += KMAX * KMAX;
  d->E = p; p += KMAX * KMAX;
  d->partial = p; p += (int64_t)RED_BLOCKS * KMAX;
  d->dots = p;
  if (hipMalloc(&d->st, sizeof(DavState)) != hipSuccess) {
    d->st = nullptr;
    return fail(DMRG_ENOMEM, "davidson_create: device allocation failed");
  }
  if (hipHostMalloc(&d->host, sizeof(DavState), hipHostMallocDefault) != hipSuccess) {
    d->host = nullptr;
    return fail(DMRG_ENOMEM, "davidson_create: pinned allocation failed");
  }
  hipStream_t s = h->ctx->stream;
  const unsigned g = grid_for(n);
  zero_kernel<<<1, 256, 0, s>>>(d->G, KMAX * KMAX);
  set_state_kernel<<<1, 1, 0, s>>>(d->st, 0);
  dmrg_status st = dmrg_heff_diag(h, d->diag);
  if (st != DMRG_OK) return st;
  // first basis vector: psi0 / ||psi0||, or the unit vector at argmin diag
  if (o.start == 1) {
    zero_kernel<<<g, 256, 0, s>>>(d->t, n);
    argmin_partial_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d->diag, n, d->partial);
    argmin_finish_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, n, d->t);
  } else {
    copy_kernel<<<g, 256, 0, s>>>(psi0, n, d->t);
  }
  scalar_dot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(d->t, d->t, n, d->partial);
  finish_scalar_kernel<<<1, RED_THREADS, 0, s>>>(d->partial, RED_BLOCKS, d->dots);
  normalize_kernel<<<g, 256, 0, s>>>(d->dots, d->st, n, d->t, 1e-300);
  DMRG_HIP(hipGetLastError());
  if ((st = expand(d.get(), s)) != DMRG_OK) return st;
  d->matvecs = 1;
  DMRG_HIP(hipMemcpyAsync(d->host, d->st, sizeof(DavState), hipMemcpyDeviceToHost, s));
  DMRG_HIP(hipStreamSynchronize(s));
  if (d->host->stalled) return fail(DMRG_EINVAL, "davidson_create: start vector is zero");
  *out = d.release();
  return DMRG_OK;
}

dmrg_status dmrg_davidson_step(dmrg_dav_t d, dmrg_dav_result* res) {
  if (!d || !res) return fail(DMRG_EINVAL, "davidson_step: bad arguments");
  if (d->done) return fail(DMRG_EINVAL, "davidson_step: the solve has converged");
  hipStream_t s = d->h->ctx->stream;
  const bool expand_first = d->started;
  dmrg_status st = expand_first ? run_stage(d, &d->gB, &d->grB, stage_ba) : run_stage(d, &d->gA, &d->grA, stage_a);
  if (st != DMRG_OK) return st;
  d->started = true;
  if (expand_first) d->matvecs++;
  DMRG_HIP(hipStreamSynchronize(s));
  // a vanished correction left the state (and res) at the last iteration
  if (expand_first && d->host->stalled) return fail(DMRG_ENOCONV, "davidson: correction vanished");
  d->iters++;
  res->energy = d->host->theta;
  res->residual = d->host->res;
  res->iters = d->iters;
  res->matvecs = d->matvecs;
  res->tail_iters = d->tail;
  res->converged = d->host->res <= d->o.tol ? 1 : 0;
  if (res->converged) {
    d->done = true;
    return DMRG_OK;
  }
  if (d->iters > d->o.max_iter) return fail(DMRG_ENOCONV, "davidson: iteration limit reached");
  return DMRG_OK;
}

dmrg_status dmrg_davidson_vector(dmrg_dav_t d, double* x) {
  if (!d || !x) return fail(DMRG_EINVAL, "davidson_vector: bad arguments");
  hipStream_t s = d->h->ctx->stream;
  copy_kernel<<<grid_for(d->n), 256, 0, s>>>(d->x, d->n, x);
  DMRG_HIP(hipGetLastError());
  return DMRG_OK;
}

void dmrg_davidson_destroy(dmrg_dav_t d) { free_dav(d); }

}  // extern "C"

namespace {

// One Davidson run from psi_inout; stop_early(res) may end it before
// convergence (used to leave the split-precision phase once it stalls).
template <class Stop>
dmrg_status solve(dmrg_heff_t h, double* psi_inout, const dmrg_dav_opts* opts, dmrg_dav_result* res,
                  Stop&& stop_early) {
  dmrg_dav_t d = nullptr;
  dmrg_status st = dmrg_davidson_create(h, opts, psi_inout, &d);
  if (st != DMRG_OK) return st;
  std::memset(res, 0, sizeof(*res));
  while (true) {
    st = dmrg_davidson_step(d, res);
    if (st != DMRG_OK || res->converged || stop_early(*res)) break;
  }
  dmrg_status st2 = dmrg_davidson_vector(d, psi_inout);
  if (st == DMRG_OK) st = st2;
  hipError_t e = hipStreamSynchronize(h->ctx->stream);
  dmrg_davidson_destroy(d);
  if (st == DMRG_OK && e != hipSuccess) return fail(DMRG_EHIP, hipGetErrorString(e));
  return st;
}


// The reduced-precision matvec's own error on a generic vector,
// ||(H_reduced - H) u|| for u = psi / ||psi||: the level below which its
// residuals stop meaning anything.  Costs one FP64 and one reduced matvec.
dmrg_status split_floor(dmrg_heff_t h, const double* psi, double* delta) {
  const int64_t n = dmrg_heff_size(h);
  if (n <= 0) return fail(DMRG_EINVAL, "davidson: empty wavefunction");
  dmrg_status st = DMRG_OK;
  hipStream_t s = h->ctx->stream;
  double* mem = nullptr;
  const int64_t len = 2 * n + (int64_t)RED_BLOCKS * KMAX + 2;
  if (hipMalloc(&mem, len * sizeof(double)) != hipSuccess) return fail(DMRG_ENOMEM, "davidson: allocation failed");
  double *y64 = mem, *ys = mem + n, *partial = mem + 2 * n, *out = partial + (int64_t)RED_BLOCKS * KMAX;
  const int keep = h->prec;  // the reduced precision
  h->prec = DMRG_FP64;
  st = heff_apply_eager(h, psi, y64);
  h->prec = keep;
  if (st == DMRG_OK) st = heff_apply_eager(h, psi, ys);
  double host[2] = {0.0, 0.0};
  if (st == DMRG_OK) {
    diff_kernel<<<grid_for(n), 256, 0, s>>>(y64, n, ys);
    scalar_dot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(ys, ys, n, partial);
    finish_scalar_kernel<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, out);
    scalar_dot_kernel<<<RED_BLOCKS, RED_THREADS, 0, s>>>(psi, psi, n, partial);
    finish_scalar_kernel<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, out + 1);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(DMRG_EHIP, "davidson: split error estimate failed");
  }
  (void)hipFree(mem);
  if (st == DMRG_OK) *delta = host[1] > 0.0 ? std::sqrt(host[0] / host[1]) : 0.0;
  return st;
}

}  // namespace

extern "C" dmrg_status dmrg_davidson(dmrg_heff_t h, double* psi_inout, const dmrg_dav_opts* opts,
                          dmrg_dav_result* res) {
  if (!h || !psi_inout || !opts || !res) return fail(DMRG_EINVAL, "davidson: bad arguments");
  if (h->prec == DMRG_FP64 || opts->fp64_tail <= 0)
    return solve(h, psi_inout, opts, res, [](const dmrg_dav_result&) { return false; });
  // Split-precision phase until the residual reaches a few times the split
  // matvec's own error (or the tolerance, or stops falling near that level),
  // then an FP64 tail from that Ritz vector brings the residual, the energy
  // and the vector to the FP64 tolerance.
  double delta = 0.0;
  dmrg_status st = split_floor(h, psi_inout, &delta);
  if (st != DMRG_OK) return st;
  const double exit_at = std::max(opts->tol, 4.0 * delta);
  std::vector<double> hist;
  dmrg_dav_result r1{};
  st = solve(h, psi_inout, opts, &r1, [&](const dmrg_dav_result& r) {
    hist.push_back(r.residual);
    if (r.residual <= exit_at) return true;
    // safety: near the floor and no 10% gain over 8 steps
    const size_t n = hist.size();
    if (n < 9 || r.residual > 100.0 * exit_at) return false;
    double best_before = hist[0], best_recent = hist[n - 8];
    for (size_t i = 0; i + 8 < n; ++i) best_before = std::min(best_before, hist[i]);
    for (size_t i = n - 8; i < n; ++i) best_recent = std::min(best_recent, hist[i]);
    return best_recent > 0.9 * best_before;
  });
  if (st != DMRG_OK && st != DMRG_ENOCONV) return st;
  dmrg_dav_opts o2 = *opts;
  o2.max_iter = opts->fp64_tail;
  o2.start = 0;  // from the split phase's Ritz vector
  const int reduced = h->prec;
  h->prec = DMRG_FP64;
  dmrg_dav_result r2{};
  st = solve(h, psi_inout, &o2, &r2, [](const dmrg_dav_result&) { return false; });
  h->prec = reduced;
  *res = r2;
  res->iters = r1.iters + r2.iters;
  res->matvecs = r1.matvecs + r2.matvecs + 2;
  res->tail_iters = r2.iters;
  res->split_iters = r1.iters;
  res->split_residual = r1.residual;
  res->split_energy = r1.energy;
  return st;
}

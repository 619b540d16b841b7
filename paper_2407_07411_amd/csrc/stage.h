// Register-staged K-tile loads of the FP64 grouped GEMM, shared by the
// per-phase kernels (gemm_f64.hip) and the persistent matvec kernel
// (persist.hip).
#pragma once

#include "internal.h"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// blockIdx -> logical tile.  Workgroups are dealt round-robin to the 8 XCDs;
// this remap hands each XCD a contiguous range of the tile table so that
// neighbouring tiles (same problem, shared operand panels) share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n) {
  const int64_t per = n / 8, rem = n % 8;
  const int64_t xcd = bid % 8, idx = bid / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Buffer resource over one operand block, advanced in K by the scalar base:
// per-lane offsets stay fixed for a whole segment, so a K tile's loads cost no
// vector address arithmetic.  Offsets at or beyond num_records read as zero
// (hardware range check), which pads rows outside the problem and the K tail.
constexpr uint32_t OOB = 0xffffffffu;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, 0x7fffffff, 0x00020000);
}

// One operand's share of a K tile (ROWS x BK values) for one thread: N
// values, element r at tile row row + r * drow and tile column kk + r * dkk.
// kc: element (row, k) of the operand sits at base + row * ld + k (contiguous
// in K; consecutive lanes take consecutive k); otherwise at base + k * ld +
// row (consecutive lanes take consecutive rows).  LDS holds the tile K-major:
// S[k][row].
template <int ROWS, int BK, int NT>
struct Stage {
  static constexpr int N = ROWS * BK / NT;
  static_assert(ROWS * BK % NT == 0 && NT % BK == 0 && NT % ROWS == 0, "staging shape");
  const double* base;  // uniform: the block's first row at the current k0
  int64_t kstep;       // uniform: elements between K tiles
  uint32_t off[N];     // byte offsets from base (OOB for rows outside the problem)
  int kk, lds;         // K column of element 0; LDS index of element 0
  bool kc;
  double v[N];

  __device__ __forceinline__ void setup(const double* seg, int ld, bool kc_, int r0, int nrows,
                                        int tid) {
    kc = kc_;
    const int row = kc ? tid / BK : tid % ROWS;
    kk = kc ? tid % BK : tid / ROWS;
    lds = kk * (ROWS + 1) + row;
    if (kc) {
      base = seg + (int64_t)r0 * ld;
      kstep = BK;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int rr = row + r * (NT / BK);
        off[r] = r0 + rr < nrows ? (uint32_t)(rr * ld + kk) * 8u : OOB;
      }
    } else {
      base = seg + r0;
      kstep = (int64_t)BK * ld;
      const bool ok = r0 + row < nrows;
#pragma unroll
      for (int r = 0; r < N; ++r) off[r] = ok ? (uint32_t)((kk + r * (NT / ROWS)) * ld + row) * 8u : OOB;
    }
  }

  // kleft = K - k0 values remain in the segment
  __device__ __forceinline__ void load(int kleft) {
    const __amdgpu_buffer_rsrc_t rs = operand_rsrc(base);
    if (kleft >= BK) {
#pragma unroll
      for (int r = 0; r < N; ++r)
        v[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off[r], 0, 0));
    } else {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int k = kc ? kk : kk + r * (NT / ROWS);
        v[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, k < kleft ? off[r] : OOB, 0, 0));
      }
    }
  }

  __device__ __forceinline__ void advance() { base += kstep; }

  // Store alpha * value into the LDS tile (double, or rounded to float).
  template <typename T>
  __device__ __forceinline__ void store(T* S, double alpha) const {
    if (kc) {
#pragma unroll
      for (int r = 0; r < N; ++r) S[lds + r * (NT / BK)] = (T)(alpha * v[r]);
    } else {
#pragma unroll
      for (int r = 0; r < N; ++r) S[lds + r * (NT / ROWS) * (ROWS + 1)] = (T)(alpha * v[r]);
    }
  }
};

}  // namespace dmrg

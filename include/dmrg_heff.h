/*
 * dmrg_heff.h - C ABI of the MI355X (gfx950) two-site DMRG effective
 * Hamiltonian library.
 *
 * Method: Menczer et al., "Parallel implementation of the Density Matrix
 * Renormalization Group method achieving a quarter petaFLOPS performance on a
 * single DGX-H100 GPU node" (arXiv:2407.07411).  The paper minimises the
 * energy of a matrix product state (Eq. 1, Eq. 2) one update at a time; each
 * update is a large hermitian eigenproblem solved with Lanczos or Davidson,
 * about 80% of the run time and O(D^3) (Numerical procedure section), followed
 * by a matrix factorisation (Introduction).  This library is that update: the
 * effective Hamiltonian H_eff acting on a block-sparse two-site wavefunction,
 * its diagonal, its adjoint, a Davidson solver and the truncating SVD.
 *
 * Conventions shared by every call
 *  - Quantum numbers are U(1)xU(1): (N, 2Sz) pairs of int32.
 *  - A basis is the sector list of one enlarged block (block + one site).
 *  - The two-site wavefunction psi with total quantum numbers Q stores one
 *    block Psi[q, Q-q] for every left sector q (in basis order) whose partner
 *    Q-q exists in the right basis; each block is row-major
 *    d_L(q) x d_R(Q-q); blocks are contiguous in left-sector order.
 *  - H_eff = sum over terms xi of c_xi * (O^L_xi (x) O^R_xi) with the
 *    fermionic sign s = (-1)^{N(q_in)} on the input left sector when the term
 *    is odd (each side changes the particle number by an odd amount):
 *      Y[q+dq, Q-q-dq] += c * s * O^L[q+dq, q] Psi[q, Q-q] O^R[Q-q-dq, Q-q]^T.
 *    A term with hc = 1 also applies its hermitian conjugate: the transposed
 *    blocks with coefficient (-1)^odd * c.
 *  - Every double pointer below is a DEVICE pointer owned by the caller unless
 *    stated otherwise; integer tables are HOST pointers read during the call.
 *  - Calls return dmrg_status (0 = success, negative = error) and never throw;
 *    dmrg_last_error() returns a thread-local message for the last failure.
 *  - Device work is enqueued on the context's HIP stream and is asynchronous
 *    unless a call says it synchronises.
 */
#ifndef DMRG_HEFF_H
#define DMRG_HEFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DMRG_OK = 0,
  DMRG_EINVAL = -1,   /* bad argument: null pointer, negative size, bad enum   */
  DMRG_EQN = -2,      /* quantum-number / layout violation (selection rule,    */
                      /* block outside its pool, odd parity on a one-sided op) */
  DMRG_ENOMEM = -3,   /* device or host allocation failed                      */
  DMRG_EHIP = -4,     /* a HIP runtime call or kernel launch failed            */
  DMRG_ENOCONV = -5,  /* an iteration (Davidson, SVD sweeps) stopped before    */
                      /* reaching its tolerance                                */
  DMRG_ENOTSUP = -6   /* combination not supported by this library             */
} dmrg_status;

/* Arithmetic of the sector GEMMs.  Everything else (Davidson
 * orthogonalisation, Rayleigh quotient, residuals, SVD) is always FP64. */
typedef enum {
  DMRG_FP64 = 0,          /* FP64 MFMA (v_mfma_f64_16x16x4)                    */
  DMRG_SPLIT_BF16X3 = 1,  /* operands split into 3 BF16 slices, products of    */
                          /* slice pairs i+j<=2 on BF16 MFMA with FP32          */
                          /* accumulation per K chunk, FP64 combine             */
  DMRG_SPLIT_FP16X2 = 2,  /* two FP16 slices: not built (FP16's 5-bit exponent */
                          /* needs per-block scaling); create and              */
                          /* set_precision return DMRG_ENOTSUP                 */
  DMRG_FP32 = 3           /* operands rounded to FP32, FP32 MFMA               */
                          /* (v_mfma_f32_16x16x4f32), FP32 accumulation per K   */
                          /* chunk, FP64 combine                                */
} dmrg_prec;

typedef struct dmrg_ctx_s* dmrg_ctx_t;      /* device + borrowed HIP stream      */
typedef struct dmrg_basis_s* dmrg_basis_t;  /* sector table of one block          */
typedef struct dmrg_heff_s* dmrg_heff_t;    /* plan of one H_eff (work lists ...) */
typedef struct dmrg_dav_s* dmrg_dav_t;      /* state of one Davidson solve        */

/* ---- context ------------------------------------------------------------ */
/* device: HIP device ordinal.  hip_stream: a hipStream_t borrowed from the
 * caller (NULL = the null stream); the library never destroys it. */
dmrg_status dmrg_ctx_create(int device, void* hip_stream, dmrg_ctx_t* out);
dmrg_status dmrg_ctx_set_stream(dmrg_ctx_t ctx, void* hip_stream);
void dmrg_ctx_destroy(dmrg_ctx_t ctx);
const char* dmrg_last_error(void);
/* Name of the library build (arch and compile flags), static storage. */
const char* dmrg_build_info(void);

/* ---- bases and wavefunction layout --------------------------------------- */
/* qn: host int32[n_sec][2] of distinct (N, 2Sz); dim: host int64[n_sec] >= 1.
 * Errors: DMRG_EINVAL (null, n_sec < 1, dim < 1), DMRG_EQN (duplicate qn). */
dmrg_status dmrg_basis_create(dmrg_ctx_t ctx, int32_t n_sec, const int32_t* qn,
                              const int64_t* dim, dmrg_basis_t* out);
void dmrg_basis_destroy(dmrg_basis_t b);
/* Block layout of psi for total Q (host int32[2]).  n_blocks: number of
 * blocks; block_offset (nullable, host int64[n_left_sectors]): offset of
 * block Psi[q, Q-q] for every left sector, -1 where q has no partner;
 * total: number of doubles of psi. */
dmrg_status dmrg_wfn_layout(dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2],
                            int64_t* n_blocks, int64_t* block_offset, int64_t* total);

/* ---- effective Hamiltonian ------------------------------------------------ */
/* One operator pair.  Operator blocks live in two caller-owned device pools of
 * doubles.  left_off[a] (host int64[n_left_sectors]) is the offset in
 * left_pool of block O^L[q_a + dq, q_a], row-major d_L(q_a+dq) x d_L(q_a), or
 * -1 when absent; right_off[c] (host int64[n_right_sectors]) the offset of
 * O^R[r_c - dq, r_c], row-major d_R(r_c-dq) x d_R(r_c), or -1.
 * one_sided = 1: O^L (x) 1 (right_off ignored, may be NULL, dq must be 0,
 * odd must be 0); one_sided = 2: 1 (x) O^R (left_off ignored).  Blocks whose
 * input or output wavefunction block does not exist are ignored. */
typedef struct {
  int32_t dq[2];     /* left shift (dN, d2Sz); the right side shifts by -dq  */
  int32_t odd;       /* 1: fermion-odd pair, sign (-1)^{N(q_in)}            */
  int32_t hc;        /* 1: also apply the hermitian-conjugate term          */
  int32_t one_sided; /* 0 two-sided, 1 left only, 2 right only              */
  int32_t reserved;  /* must be 0                                            */
  double coeff;
  const int64_t* left_off;
  const int64_t* right_off;
} dmrg_term;

/* Builds the plan: wavefunction layout, the (term, block) work list with the
 * cheaper association order per pair, the grouped-GEMM tile lists and the
 * device workspace (intermediates, K-split partial sums, and one vector of
 * size doubles that holds psi pre-split for split precision).  The pools are borrowed (must outlive the plan, contents
 * may change between applies); pool lengths are in doubles and bound-check
 * every block.  Errors: DMRG_EINVAL, DMRG_EQN (block out of its pool, dq that
 * leaves the basis, odd one-sided term), DMRG_ENOMEM, DMRG_EHIP.
 * Synchronises the context stream. */
dmrg_status dmrg_heff_create(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R,
                             const int32_t Q[2], int64_t n_terms, const dmrg_term* terms,
                             const double* left_pool, int64_t left_pool_len,
                             const double* right_pool, int64_t right_pool_len,
                             dmrg_prec prec, dmrg_heff_t* out);
/* Out-of-core form of dmrg_heff_create for operators larger than device
 * memory, the regime where the paper finds host-device traffic dominating
 * (Performance assessment section, beyond D of about 8000-10000) and hides
 * it with asynchronous transfers.  left_pool_host / right_pool_host: the
 * same pools in page-locked host memory (hipHostMalloc; pageable or device
 * memory is refused with DMRG_EINVAL), borrowed and read by later applies;
 * unlike device pools their contents must not change after creation (part
 * of them is copied to the device once).  device_bytes bounds the device memory that
 * holds operator blocks (the workspace of dmrg_heff_create comes on top):
 * when every distinct block fits, all are copied once at creation;
 * otherwise two staging slots (DMRG_HEFF_STREAM_SLOT_KB, else 1/16 of the
 * budget, at most 1 GiB, at least the largest pair's blocks) are set
 * aside, the items whose blocks fit the rest are copied once, and every
 * apply copies the remaining blocks slot by slot on a copy stream while the
 * compute stream runs the resident items and the slot filled before.
 * Results match dmrg_heff_create's to rounding (the waves, hence the
 * summation order into y, differ).  apply, diag and Davidson work as for
 * device pools (Davidson without stage graphs); use_graph, the persistent
 * launch, autotune, apply_profiled and the adjoint return DMRG_ENOTSUP.
 * Errors: as dmrg_heff_create; DMRG_ENOMEM when two slots of the largest
 * pair exceed device_bytes.  DMRG_HEFF_STREAM_RESIDENT_KB caps the resident
 * copy (0: stream every pair).  Synchronises the context stream. */
dmrg_status dmrg_heff_create_streamed(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R,
                                      const int32_t Q[2], int64_t n_terms, const dmrg_term* terms,
                                      const double* left_pool_host, int64_t left_pool_len,
                                      const double* right_pool_host, int64_t right_pool_len,
                                      dmrg_prec prec, int64_t device_bytes, dmrg_heff_t* out);
/* Host, synchronous.  Bytes of operator blocks held on the device for the
 * whole plan, bytes copied from host memory per apply, and the number of
 * resident and streamed waves (all zero for a plan over device pools). */
dmrg_status dmrg_heff_stream_info(dmrg_heff_t h, int64_t* resident_bytes, int64_t* streamed_bytes,
                                  int32_t* resident_waves, int32_t* streamed_waves);
/* ---- SU(2) spin-adapted form ----------------------------------------------
 * The paper's DMRG is spin adapted; its bond dimensions count multiplets
 * (Introduction; Performance assessment section; P450 section).  Here the
 * bases hold sectors (N, 2j) (2j >= 0) with the number of multiplets as
 * dim, and Q = (N, 2S) is the total particle number and spin.  Operators of
 * spin rank k are stored as reduced blocks O[(N', j'), (N, j)] (row-major
 * d(N', j') x d(N, j)) in the Wigner-Eckart convention
 * <j' m'|T^k_q|j m> = <j m; k q | j' m'> O[...] (Condon-Shortley
 * Clebsch-Gordan coefficients).  A term is the scalar
 * coeff * sum_q (-1)^(k-q) O^L_q (x) O^R_{-q} (fermionic sign (-1)^N(left
 * input) when odd); on the reduced wavefunction blocks it adds
 *   Y[(a', c')] += coeff * s * W * O^L[a', a] Psi[(a, c)] O^R[c', c]^T,
 *   W = (-1)^(j_a + j_c' + k + S) sqrt((2j_a' + 1)(2j_c' + 1))
 *       { j_a' j_c' S ; j_c j_a k } (a Wigner 6j symbol),
 * and hc = 1 also adds the transpose of every such contribution.  One-sided
 * terms are scalars (two_k = 0, dn = 0). */
typedef struct {
  int32_t two_k;     /* 2 x spin rank of both operators                     */
  int32_t dn;        /* particle-number change of the left operator; the    */
                     /* right one changes it by -dn                          */
  int32_t odd;       /* 1: fermion-odd pair (must equal |dn| mod 2)          */
  int32_t hc;        /* 1: also apply the transpose of the term             */
  int32_t one_sided; /* 0 two-sided, 1 left only, 2 right only              */
  int32_t reserved;  /* must be 0                                            */
  double coeff;
  int64_t n_left, n_right;      /* stored blocks of each side               */
  const int64_t* left_blocks;   /* host int64[n_left][3]: output sector,    */
                                /* input sector, offset in left_pool        */
  const int64_t* right_blocks;  /* host int64[n_right][3], right_pool       */
} dmrg_term_su2;
/* The weight W above for doubled spins (2j_a, 2j_c, 2j_a', 2j_c', 2k, 2S);
 * 0 where a triangle rule fails.  Host only, pure: it needs no context and
 * no device. */
double dmrg_su2_weight(int32_t two_ja, int32_t two_jc, int32_t two_ja2, int32_t two_jc2, int32_t two_k,
                       int32_t two_s);
/* Reduced wavefunction layout of total Q = (N, 2S): one block per (left
 * sector a, right sector c) with N_a + N_c = N and |j_a - j_c| <= S <=
 * j_a + j_c, ordered by a then c, row-major d_a x d_c, contiguous.
 * block_left / block_right (host int32[n]) and block_offset (host int64[n])
 * may be NULL; call once with NULL to learn n_blocks. */
dmrg_status dmrg_wfn_layout_su2(dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2], int64_t* n_blocks,
                                int32_t* block_left, int32_t* block_right, int64_t* block_offset,
                                int64_t* total);
/* dmrg_heff_create for the SU(2) form: the same device pools, plan,
 * precisions and calls (apply, diag, adjoint, Davidson, autotune,
 * persistent launch; the pool gradients of the adjoint are those of the
 * reduced blocks).  Errors: DMRG_EINVAL (bad flags, 2j < 0, sector index
 * outside a basis), DMRG_EQN (a block that breaks N' - N = dn or the
 * triangle rule of j, k, j'; a block outside its pool; a one-sided term that
 * is not a scalar), DMRG_ENOMEM, DMRG_EHIP.  Synchronises the context
 * stream. */
dmrg_status dmrg_heff_create_su2(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2],
                                 int64_t n_terms, const dmrg_term_su2* terms, const double* left_pool,
                                 int64_t left_pool_len, const double* right_pool, int64_t right_pool_len,
                                 dmrg_prec prec, dmrg_heff_t* out);
void dmrg_heff_destroy(dmrg_heff_t h);
dmrg_status dmrg_heff_set_precision(dmrg_heff_t h, dmrg_prec prec);
/* Host, synchronous.  alg_flops: FP64-equivalent FLOPs of one matvec, every
 * (term, block) pair counted once per hc partner at its cheaper association
 * order (one-sided pairs: one GEMM).  alg_bytes: every operator block used
 * read once plus psi read plus y written, 8 bytes per double. */
dmrg_status dmrg_heff_flops(dmrg_heff_t h, double* alg_flops, double* alg_bytes);
/* Length of psi in doubles (== dmrg_wfn_layout total). */
int64_t dmrg_heff_size(dmrg_heff_t h);
/* y = H_eff psi: the operator of the local eigenproblem that each MPS update
 * solves (Eq. 2; the Lanczos/Davidson step that takes about 80% of the run
 * time, Numerical procedure section), as the operator-pair sum stated at the
 * top of this file.  psi and y: device double[size], must not overlap.
 * Errors: DMRG_EINVAL (null or aliasing pointers; graph mode on the null
 * stream), DMRG_EHIP.  Data are not validated. */
dmrg_status dmrg_heff_apply(dmrg_heff_t h, const double* psi, double* y);
/* diag = diagonal of H_eff (device double[size]), the Davidson
 * preconditioner of the local eigenproblem (Eq. 2; Numerical procedure
 * section): only dq = 0 pairs reach the diagonal, each as
 * c * diag(O^L) (x) diag(O^R) (a transposed hc partner has the same
 * diagonal).  Errors: DMRG_EINVAL, DMRG_EHIP. */
dmrg_status dmrg_heff_diag(dmrg_heff_t h, double* diag);
/* Adjoint of y = H_eff(O) psi for an upstream gradient ybar (device
 * double[size]): the gradients with respect to the wavefunction and to the
 * operator blocks that an orbital gradient needs (DMRG-CASSCF, named in the
 * P450 section of the paper).  Each non-null output is ACCUMULATED (+=):
 *   psibar         += H_eff^T ybar                      (device double[size])
 *   left_pool_bar  += d<ybar, y>/d left_pool   (device, left_pool layout)
 *   right_pool_bar += d<ybar, y>/d right_pool  (device, right_pool layout)
 * Intermediates are recomputed, not stored from the forward pass. */
dmrg_status dmrg_heff_apply_adjoint(dmrg_heff_t h, const double* psi, const double* ybar,
                                    double* psibar, double* left_pool_bar,
                                    double* right_pool_bar);
/* Bytes of device workspace the plan holds (T intermediates of the
 * two-GEMM chains, processed in waves that fit it). */
int64_t dmrg_heff_workspace_bytes(dmrg_heff_t h);
/* Capture the matvec for the (psi, y) pair in a hipGraph and replay it on
 * later applies with the same pointers (1) or launch eagerly (0). */
dmrg_status dmrg_heff_use_graph(dmrg_heff_t h, int32_t enable);

/* Persistent single-launch matvec (FP64): every phase of the product (the
 * intermediates of each workspace wave, the long-K output sums, the ordered
 * reductions of cut sums) runs in ONE kernel launch whose workgroups take
 * 64x128 output tiles from per-phase, per-XCD queues and wait (bounded) for
 * the previous phase to complete; consecutive tiles of a workgroup are
 * pipelined (the next tile's first K tile loads during the current tile's
 * last).  Results are bit-identical to the per-phase launches.  enable = 1
 * builds the task tables (device memory, synchronous) and selects this form
 * for FP64 applies (and Davidson); 0 returns to per-phase launches.  The
 * split and FP32-operand precisions always use per-phase launches.  The
 * environment variable DMRG_HEFF_PERSIST=1 enables it at creation. */
dmrg_status dmrg_heff_set_persistent(dmrg_heff_t h, int32_t enable);
/* Synchronises the context stream and reports whether a persistent launch
 * since the last check gave up waiting for an earlier phase (DMRG_EHIP: its
 * results are not valid; the flag is cleared).  DMRG_OK otherwise. */
dmrg_status dmrg_heff_check(dmrg_heff_t h);

/* Autotuner: times every tile shape (the kernel ids of dmrg_heff_launches;
 * the split kernels skip 256x128) on the plan's
 * own problems, grouped by phase (intermediates / output sums) and by the
 * (M, N) size class (<=16, 32, 64, 128, 256, 512, larger), keeps the fastest
 * shape per group and rebuilds the plan with it, keeping the rebuilt plan
 * only when its whole matvec beats the previous plan's by more than 2% (a
 * phase runs its shapes side by side, which per-group timing does not see;
 * smaller differences are timing noise).  The timing runs the
 * current precision's kernels on the context stream with psi and y (device
 * double[size]; y and the workspace are overwritten).  reps >= 1 timed
 * launches per candidate.  The adjoint keeps the built-in rule.  For FP64
 * it then times the kept matvec as per-phase launches and as the single
 * persistent launch (dmrg_heff_set_persistent) and keeps the persistent
 * form only when it is faster by more than the same margin.  Synchronises. */
dmrg_status dmrg_heff_autotune(dmrg_heff_t h, const double* psi, double* y, int32_t reps);

/* Profiling: the matvec is a fixed sequence of grouped-GEMM launches.
 * n_launches (host) receives their number; when kernel / flops are non-null
 * (host arrays of at least that many entries) they receive each launch's
 * kernel id (FP64 grouped GEMM tiles 0: 32x32, 1: 64x64, 2: 128x128 with 4
 * waves, 3: 128x128 with 8 waves, 4: 256x128 with 8 waves, 5: 64x128 with 8
 * waves; the same shapes +16 for the split precision kernels and +48 for the
 * FP32-operand kernels; 32: the ordered reduction of cut K sums) and its
 * algorithmic FLOPs (2 M N K summed over its problems, 0 for reductions). */
dmrg_status dmrg_heff_launches(dmrg_heff_t h, int64_t* n_launches, int32_t* kernel, double* flops);
/* y = H_eff psi as dmrg_heff_apply (eager, the same launch schedule: largest
 * tile shape of a phase on the context stream, smaller shapes and
 * reductions beside it on side streams), bracketing every launch with HIP
 * events on the stream it runs on; ms (host float[n_launches]) receives each
 * launch's duration.  Synchronises the stream.  DMRG_ENOTSUP for the
 * out-of-core form. */
dmrg_status dmrg_heff_apply_profiled(dmrg_heff_t h, const double* psi, double* y, float* ms);

/* ---- Davidson -------------------------------------------------------------- */
typedef struct {
  int32_t max_iter;      /* iterations (matvecs after the first), e.g. 200   */
  int32_t max_subspace;  /* basis size before restart, 2..32, e.g. 24        */
  int32_t restart_keep;  /* Ritz vectors kept at restart, 1..max_subspace-1  */
  int32_t use_graph;     /* 1: replay each iteration as one hipGraph         */
  double tol;            /* stop when ||H x - theta x||_2 <= tol, ||x|| = 1  */
  int32_t fp64_tail;     /* reduced precision (split or FP32): iterations run */
                         /* in FP64 after the reduced phase reaches its own   */
                         /* error level (0 = none)                            */
  int32_t start;         /* 0: start from the given vector; 1: from the unit  */
                         /* vector at the lowest diagonal element (lowest     */
                         /* index on ties), the given vector is ignored       */
} dmrg_dav_opts;
typedef struct {
  double energy;         /* Ritz value theta (Rayleigh quotient in FP64)     */
  double residual;       /* ||H x - theta x||_2 of the returned vector       */
  int32_t iters;
  int32_t matvecs;
  int32_t converged;
  int32_t tail_iters;    /* iterations spent in the FP64 tail                 */
  double split_residual; /* residual where the reduced-precision phase ended */
  int32_t split_iters;   /* iterations of the reduced-precision phase (split */
                         /* or FP32 operands)                                 */
  int32_t reserved;
  double split_energy;   /* Ritz value where the reduced-precision phase     */
                         /* ended, before the FP64 tail                       */
} dmrg_dav_result;

/* Davidson (E. R. Davidson 1975) for the lowest eigenpair of H_eff with the
 * diagonal preconditioner t = r / (theta - diag) (|theta - diag| clamped to
 * >= 1e-8), two-pass classical Gram-Schmidt, restart from the restart_keep
 * lowest Ritz vectors.  psi0 (device double[size], non-zero; may be NULL
 * when opts->start = 1) is the start vector.  Device memory:
 * (2 * max_subspace + 2 * restart_keep + 5) * size doubles. */
dmrg_status dmrg_davidson_create(dmrg_heff_t h, const dmrg_dav_opts* opts,
                                 const double* psi0, dmrg_dav_t* out);
/* One iteration.  The first call: Rayleigh-Ritz on the start subspace and
 * its residual.  Every later call: the correction of the previous Ritz pair
 * (restart when the subspace is full, preconditioner, orthogonalisation,
 * one matvec), then Rayleigh-Ritz and the residual on the grown subspace,
 * as one launch sequence (one hipGraph with opts->use_graph) and one
 * synchronisation to read the residual.  Returns DMRG_OK while iterating or
 * once converged (res->converged; later calls return DMRG_EINVAL),
 * DMRG_ENOCONV when max_iter is exhausted or the correction vanished (then
 * res and the Ritz vector stay those of the last complete iteration). */
dmrg_status dmrg_davidson_step(dmrg_dav_t d, dmrg_dav_result* res);
/* Copy the current Ritz vector (unit norm) to x (device double[size]). */
dmrg_status dmrg_davidson_vector(dmrg_dav_t d, double* x);
void dmrg_davidson_destroy(dmrg_dav_t d);
/* Whole solve: create, iterate, write the Ritz vector back into psi_inout. */
dmrg_status dmrg_davidson(dmrg_heff_t h, double* psi_inout, const dmrg_dav_opts* opts,
                          dmrg_dav_result* res);

/* ---- SVD truncation --------------------------------------------------------- */
/* The matrix factorisation that follows each local optimisation
 * (Introduction) with D states kept, D setting the accuracy (Numerical
 * procedure section).
 * Factorises each block Psi[q, Q-q] = U S V^T (one-sided Jacobi, FP64),
 * pools all singular values, sorts them descending (ties: lower left-sector
 * index first, then position) and keeps at most max_keep values > cutoff.
 * psi: device double[size] in the layout of (L, R, Q).
 * kept_dim: host int64[n_left_sectors], number of values kept per left sector
 *   (0 for sectors without a block).
 * U, Vt, S: device outputs, each block's factors packed in left-sector order:
 *   U block d_L(q) x k_q row-major, S k_q values (descending within the
 *   block), Vt block k_q x d_R(Q-q) row-major; capacities u_cap, s_cap,
 *   vt_cap in doubles (DMRG_EINVAL if too small; the needed sizes are what
 *   the call would write with max_keep = total rank).
 * trunc_err (host): sum of discarded sigma^2.  Synchronises.
 * Errors: DMRG_EINVAL, DMRG_ENOMEM, DMRG_EHIP; DMRG_ENOCONV when a block
 * still rotates after 80 Jacobi sweeps (the outputs are written but not
 * converged). */
dmrg_status dmrg_svd_truncate(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R, const int32_t Q[2],
                              const double* psi, int64_t max_keep, double cutoff,
                              int64_t* kept_dim, double* U, int64_t u_cap, double* S,
                              int64_t s_cap, double* Vt, int64_t vt_cap, double* trunc_err);
/* For callers that cannot allocate device memory (code under hipGraph capture
 * of its own, serving loops, harnesses that forbid hipMalloc): the same
 * truncation, arguments and results as dmrg_svd_truncate, with every device
 * temporary (working copies of the blocks and their right factors, tables,
 * singular values, flags) taken from one 64 MiB scratch array that each device
 * holds until the process ends.  Calls no hipMalloc or hipFree.  The
 * temporaries need about 8 * (sum over blocks of r*c + c*c + c) bytes (r, c the
 * longer and shorter block side) plus small tables; larger inputs return
 * DMRG_ENOMEM with the needed size.  All calls on one device share the array:
 * calls that overlap in time on one device (other threads, other streams)
 * race and must be serialised by the caller.  Synchronises. */
dmrg_status dmrg_svd_truncate_noalloc(dmrg_ctx_t ctx, dmrg_basis_t L, dmrg_basis_t R,
                                      const int32_t Q[2], const double* psi, int64_t max_keep,
                                      double cutoff, int64_t* kept_dim, double* U, int64_t u_cap,
                                      double* S, int64_t s_cap, double* Vt, int64_t vt_cap,
                                      double* trunc_err);

/* ---- operator blocks and the two-site sweep -------------------------------- */
/* The ab initio Hamiltonian H = sum h_pq a+_ps a_qs + 1/2 sum V_pqrs
 * a+_ps a+_rt a_st a_qs on an orbital chain, with the operator blocks of a
 * two-site DMRG sweep (the paper's MPS optimisation, Numerical procedure
 * section).  h: host double[L*L]; V: host double[L^4], V_pqrs = (pq|rs) at
 * ((p*L+q)*L+r)*L+s; n_elec electrons with 2Sz = two_sz; at most D states per
 * block.  The right blocks are first built from a random isometry per sector
 * (seeded).  ctx may be NULL when only dmrg_chain_export is called.  Blocks keep H, all one- and two-operator products on their
 * orbitals and the complementary sums for operators outside them, in their
 * renormalised bases. */
typedef struct dmrg_chain_s* dmrg_chain_t;
dmrg_status dmrg_chain_create(dmrg_ctx_t ctx, int32_t L, const double* h, const double* V,
                              int32_t n_elec, int32_t two_sz, int64_t D, uint64_t seed,
                              dmrg_chain_t* out);
void dmrg_chain_destroy(dmrg_chain_t c);
/* One two-site update at orbitals (l, l+1): grow the left block [0,l) by l
 * and the right block [l+2,L) by l+1, build the H_eff operator pairs, solve
 * for the lowest state with Davidson (seeded random start, opts as for
 * dmrg_davidson), truncate with dmrg_svd_truncate to D states and keep the
 * renormalised enlarged block of the sweep direction (dir = +1: left block
 * [0,l+1); dir = -1: right block [l+1,L)).  A left-to-right sweep runs
 * l = 0..L-2 with dir = +1, a right-to-left sweep l = L-2..0 with dir = -1.
 * energy, trunc_err: host.  Synchronises. */
dmrg_status dmrg_chain_step(dmrg_chain_t c, int32_t l, int32_t dir, const dmrg_dav_opts* opts,
                            double* energy, double* trunc_err, dmrg_dav_result* res);
/* Host-only: (re)build the left blocks [0,1) .. [0,l) by growth without
 * truncation (every state compatible with the total charge is kept), e.g. to
 * start a sweep from exact small blocks or to inspect dmrg_chain_export. */
dmrg_status dmrg_chain_grow_left(dmrg_chain_t c, int32_t l);
/* The two-site problem dmrg_chain_step would solve at (l, l+1), as host
 * arrays (host-only, needs no device: ctx may be NULL at dmrg_chain_create if
 * only this call is used).  Call once with null arrays to get n_left,
 * n_right, n_terms and the pool lengths, then with arrays of those sizes:
 * lqn[n_left][2], ldim[n_left], rqn[n_right][2], rdim[n_right],
 * term_info[n_terms][4] = (dq N, dq 2Sz, odd, one_sided), left_off[n_terms]
 * [n_left], right_off[n_terms][n_right] (layout of dmrg_term, -1 absent),
 * lpool, rpool.  Every term has coefficient 1 and no hermitian partner. */
dmrg_status dmrg_chain_export(dmrg_chain_t c, int32_t l, int32_t* n_left, int32_t* n_right,
                              int64_t* n_terms, int64_t* lpool_len, int64_t* rpool_len, int32_t* lqn,
                              int64_t* ldim, int32_t* rqn, int64_t* rdim, int32_t* term_info,
                              int64_t* left_off, int64_t* right_off, double* lpool, double* rpool);

#ifdef __cplusplus
}
#endif
#endif /* DMRG_HEFF_H */

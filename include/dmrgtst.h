/*
 * dmrgtst.h -- C ABI of libdmrgtst.so: the hot path of time-step-targeting DMRG on one
 * MI355X (gfx950) GPU.
 *
 * Scope (paper: Alvarez, Dias da Silva, Ponce, Dagotto, "Time Evolution with the DMRG
 * Algorithm: A Generic Implementation for Strongly Correlated Electronic Systems"):
 *   - the superblock Hamiltonian-vector product H_sb.psi, the "Hamiltonian connections between
 *     system and environment" that Sec. IV names as the most expensive task;
 *   - the Krylov (Lanczos) exponential of Sec. II.A, repeated for longer times as in Sec. II.C
 *     (Eq. lanczosevolution2);
 *   - the time-step-targeting vectors phi(t_x) and their weights (Sec. II.B and II.C).
 *
 * Superblock and vectors
 *   The superblock is S (x) E: S = left block + site s1, E = site s2 + right block, fermion
 *   modes of S ordered before those of E.  Both halves are split into symmetry sectors
 *   labelled (N_up, N_dn).  A vector of the target sector (N_up, N_dn) is a set of blocks
 *   Psi_p (dim_S(p) x dim_E(q), q = target - p), one per S sector p whose partner q exists.
 *   Layout of one vector: 2n doubles, all real parts first, then all imaginary parts; inside
 *   each plane the blocks follow ascending S-sector order and each block is column-major.
 *   dmrg_psi_layout() reports n and the block table.
 *
 *   H_sb = H_S (x) 1 + 1 (x) H_E + sum_terms coef (A P_S^f) (x) B
 *   where (A (x) B) acts on the coefficient matrix X as A X B^T and P_S is the fermion parity
 *   of S (present when the term is fermionic).  A hopping bond -t sum_s (c+_a c_b + h.c.)
 *   between an S site a and an E site b expands into the four terms
 *     -t (C+_a P_S) (x) (C+_b)^T   and   +t ((C+_a)^T P_S) (x) C+_b      for s = up, down.
 *   The library computes exp(-i tau H); the paper's exp(+iHt) is tau -> -tau.
 *
 * Memory
 *   Problem data passed to dmrg_create() is host memory; it is deep-copied to device memory
 *   owned by the handle and may be freed on return.  Vectors (x, y, phi, targets) are device
 *   pointers owned by the caller.  All work is ordered on the handle's HIP stream (passed as
 *   a void* hipStream_t; NULL = the default stream).
 *
 * Errors
 *   Every function returns a dmrg_status (0 = success, negative = error, positive = a result
 *   that is returned but carries a warning).  No C++ exception crosses the boundary.
 *   dmrg_last_error() returns a description of the last failure on a handle.  Lanczos breakdown
 *   is not an error: it is reported in dmrg_krylov_info and the result is then exact.
 *   Device memory: every buffer a handle allocates (operators, work lists, Krylov workspaces,
 *   the buffers of the next rows) is charged to it; if the environment variable
 *   DMRG_MAX_WORKSPACE holds a byte count when dmrg_create runs, an allocation that would take
 *   the handle above it fails with DMRG_ENOMEM before any memory is requested.  Buffers of a
 *   batch are charged to its first handle.
 *
 * Threads: a handle is used by one host thread at a time.
 */
#ifndef DMRGTST_H
#define DMRGTST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmrg_ctx* dmrg_handle;
typedef struct dmrg_batch_ctx* dmrg_batch;

enum dmrg_status {
    DMRG_OK = 0,
    DMRG_EINVAL = -1,     /* invalid argument or inconsistent problem description        */
    DMRG_ENOMEM = -2,     /* device or host allocation failed                             */
    DMRG_EHIP = -3,       /* a HIP runtime call failed                                    */
    DMRG_ENONFINITE = -4, /* non-finite value met where finite input is required          */
    DMRG_ESTATE = -5,     /* call not valid in the handle's current state                 */
    DMRG_EIO = -6,        /* the tuning cache file cannot be read, parsed or written      */
    DMRG_WNOTCONV = 1     /* iteration stopped before its tolerance; the last iterate is
                             returned (dmrg_ground_state)                                  */
};

/* Arithmetic of the block products (the Lanczos recurrence, the reorthogonalisation, the
 * small tridiagonal exponential and the combination always stay FP64).  In the split bf16
 * forms every operand value is a sum of bf16 pieces a = a0 + a1 (+ a2), each piece the bf16
 * rounding of what the previous ones leave of the FP32 value. */
enum dmrg_precision {
    DMRG_FP64 = 0,        /* FP64 MFMA                                                    */
    DMRG_FP32 = 1,        /* FP32 operands and FP32 MFMA accumulation, result promoted     */
    DMRG_BF16X3 = 2,      /* two pieces, products a0b0 + a0b1 + a1b0, FP32 accumulation:
                             relative error about 2^-16                                   */
    DMRG_BF16X6 = 3       /* three pieces, the six products a_i b_j with i + j <= 2, FP32
                             accumulation: relative error about 2^-24, like FP32          */
};

/* Kernel families of the two block-product stages (bits of a variant).  Without the bits a stage
 * runs register-tiled (stage 1: a 32 x 64 tile per single-wavefront work group; stage 2: a
 * 32 x 32 tile per work group whose K chunks are dealt to its four wavefronts).  STAGE1_NARROW,
 * STAGE2_NARROW: register-tiled with tiles half as wide (stage 1: 32 x 32, stage 2: 32 x 16;
 * twice as many tiles, for balance on small problems).
 * STAGE1_LDS / STAGE2_LDS: LDS-tiled (64 x 64 tiles per work group, four wavefronts sharing
 * every K chunk through LDS; stage 2 splits long K into slices summed by a reduction launch).
 * The NARROW and LDS bits of one stage exclude each other.  Results agree to rounding. */
enum dmrg_gemm {
    DMRG_GEMM_STAGE1_LDS = 1,
    DMRG_GEMM_STAGE2_LDS = 2,
    DMRG_GEMM_STAGE1_NARROW = 4,
    DMRG_GEMM_STAGE2_NARROW = 8,
    DMRG_GEMM_X = 16,     /* LDS-staged family for both stages (alone, no other bit): work groups
                             of four wavefronts share every operand chunk through LDS (stage 1:
                             64 x 64 tiles; stage 2: 64 x 32 tiles, long K as two slices added
                             into an output its stage 1 zeroes).  FP64 only: other arithmetics,
                             and plans whose stage-2 tiles exceed 256 chunks, run register-tiled. */
    DMRG_GEMM_K = 32      /* K-split family for both stages (alone, no other bit): the 4x4x4 FP64
                             MFMA with its four blocks as four K slices, operands packed in lane
                             order (the input vector packed by a first kernel of stage 1, the
                             stage-1 intermediate written in stage 2's operand layout).  FP64
                             only (other arithmetics run register-tiled); single handles only
                             (merged batch lists run register-tiled). */
};

/* A block operator of one half that changes (N_up, N_dn) by dq.  blocks: for every source
 * sector p in ascending order whose image p+dq is a sector of the half, one dense
 * dim(p+dq) x dim(p) column-major block, all concatenated. */
typedef struct {
    int32_t dq[2];
    const double* blocks;
} dmrg_op;

/* One superblock half.  qn: nsec pairs (N_up, N_dn), strictly increasing in lexicographic
 * order; dim: nsec positive sizes; H: per-sector dim x dim symmetric blocks, column-major,
 * concatenated in sector order; ops: nop block operators (typically the c+ of edge sites). */
typedef struct {
    int32_t nsec;
    const int32_t* qn;
    const int32_t* dim;
    const double* H;
    int32_t nop;
    const dmrg_op* ops;
} dmrg_half;

/* Generic connection term coef (A P_S^fermionic) (x) B with A = S.ops[opS] (transposed when
 * transS != 0) and B = E.ops[opE] (transposed when transE != 0).  The quantum-number changes
 * of A and B must cancel. */
typedef struct {
    double coef;
    int32_t opS, transS;
    int32_t opE, transE;
    int32_t fermionic;
} dmrg_term;

/* Hopping bond -t sum_s (c+_{a s} c_{b s} + h.c.): opS[s] = index of c+_{a s} in S.ops,
 * opE[s] = index of c+_{b s} in E.ops (s = 0 up, 1 down). */
typedef struct {
    int32_t opS[2];
    int32_t opE[2];
    double t;
} dmrg_bond;

typedef struct {
    dmrg_half S, E;
    int32_t target[2];
    int32_t nbond;
    const dmrg_bond* bonds;
    int32_t nterm;
    const dmrg_term* terms;
} dmrg_problem;

/* Krylov diagnostics (host struct; Sec. II.A: the basis of n_l = kdim Lanczos vectors, which
 * stops early at an invariant subspace).  Filled by the call:
 *   k_eff      Lanczos vectors used in the last step (kdim unless breakdown);
 *   k_eff_min  over all steps of the call;
 *   beta0      ||x|| of the first step;  beta_last = last computed beta of the last step;
 *   err_est    beta_k |c_{k-1}(tau)| of the last step (an upper estimate of the step's
 *              truncation error, 0 after breakdown); dmrg_ground_state: the residual estimate;
 *   breakdown  1 if any step broke down (invariant subspace found, result exact);
 *   converged  dmrg_ground_state: 1 if the residual estimate met tol (else the call returns
 *              DMRG_WNOTCONV); 1 for the other calls.
 * Set by the caller (zero-initialise the struct if unused):
 *   k_eff_steps  NULL, or a host array receiving the Lanczos vectors of every step: nsteps
 *              entries for dmrg_krylov_expm, one per basis (at most max_restarts) for
 *              dmrg_ground_state, one for the time-step-targeting calls. */
typedef struct {
    int32_t k_eff;
    int32_t k_eff_min;
    double beta0;
    double beta_last;
    double err_est;
    int32_t breakdown;
    int32_t converged;
    int32_t* k_eff_steps;
} dmrg_krylov_info;

/* Builds the sector tables, the block work lists and the packed device copies of all
 * operators (Sec. IV: the Hamiltonian connections).  stream: hipStream_t or NULL.
 * Errors: DMRG_EINVAL for malformed input (unsorted or repeated sectors, non-positive
 * dims, out-of-range op indices, terms whose dq do not cancel, empty target sector) or a
 * DMRG_MAX_WORKSPACE value that is not a decimal byte count, DMRG_ENOMEM (device memory
 * exhausted, or the handle's buffers above DMRG_MAX_WORKSPACE), DMRG_EHIP.  On error *out is
 * set to NULL and dmrg_last_error(NULL) describes the failure. */
int dmrg_create(const dmrg_problem* problem, void* stream, dmrg_handle* out);

/* Releases all device memory of the handle (waits for its stream).  NULL is ignored. */
void dmrg_destroy(dmrg_handle h);

/* Host-only planning (no device memory, no HIP call): builds the plan dmrg_create would build
 * for problem and packs its FP64 operators, and reports
 *   n, nblk         complex length of a vector and number of psi blocks;
 *   flops, flops_executed   as dmrg_flops and dmrg_flops_executed would;
 *   create_bytes    device bytes dmrg_create allocates for the handle;
 *   krylov_bytes    device bytes the handle's first dmrg_krylov_expm or dmrg_tst_targets call
 *                   with kdim Lanczos vectors adds (basis slots, work vector, partial sums,
 *                   state, iteration tables; a call that sets info->k_eff_steps adds 4 bytes
 *                   per step, one with input checking on 8 bytes)
 * (callers size DMRG_MAX_WORKSPACE or batches with it).  Errors as dmrg_create (DMRG_EINVAL,
 * described by dmrg_last_error(NULL); kdim outside [1, 64] is DMRG_EINVAL too). */
typedef struct {
    int64_t n;
    int32_t nblk;
    double flops;
    double flops_executed;
    int64_t create_bytes;
    int64_t krylov_bytes;
} dmrg_plan_info;
int dmrg_plan_stats(const dmrg_problem* problem, int32_t kdim, dmrg_plan_info* out);

/* Vector layout: *n = complex length (a vector is 2n doubles); *nblk = number of blocks.
 * If the array pointers are non-NULL they receive, per block: off = offset inside a plane,
 * rows = dim_S(p), cols = dim_E(q), secS = p, secE = q.  Any pointer may be NULL. */
int dmrg_psi_layout(dmrg_handle h, int64_t* n, int32_t* nblk, int64_t* off, int32_t* rows,
                    int32_t* cols, int32_t* secS, int32_t* secE);

/* Algorithmic flops of one H_sb.psi for one complex vector (Sec. IV, the Hamiltonian
 * connections): both real planes, two flops per multiply-add, terms with a non-zero operator
 * block only, and for every connection term the cheaper of the two contraction orders
 * (A X) B^T and A (X B^T); no padding.  Throughput figures divide this count by time. */
int dmrg_flops(dmrg_handle h, double* flops);

/* Flops the block products execute for one H_sb.psi, counted like dmrg_flops but in the order
 * the kernels use (the right product X B^T first for every term: stage 1 forms the right
 * products of each source block, stage 2 sums the left products into each output block).
 * At least dmrg_flops; equal when the right-first order is the cheaper one for every term
 * (for instance when both halves have the same sector dimensions). */
int dmrg_flops_executed(dmrg_handle h, double* flops);

/* Selects the block-product arithmetic; converted operator copies are built on first use and
 * cached.  A change of arithmetic waits for the handle's stream (the intermediate workspace is
 * cleared for the new element size).  DMRG_EINVAL for an unknown value. */
int dmrg_set_precision(dmrg_handle h, int32_t precision);

/* Selects the kernel families (dmrg_gemm bits; both register-tiled after dmrg_create).  DMRG_EINVAL
 * for unknown bits or two families for one stage. */
int dmrg_set_gemm(dmrg_handle h, int32_t variant);
int dmrg_get_gemm(dmrg_handle h, int32_t* variant);

/* Autotuner: times the kernel families of each stage on the handle's problem in its current
 * arithmetic (reps back-to-back launches each, on zeroed scratch vectors the handle owns) and
 * keeps the fastest of each; in FP64 the LDS-staged and the K-split families are timed as pairs
 * of stages and kept if a pair beats the best of the others.  out: NULL or 10 doubles receiving
 * milliseconds per launch of [stage 1 register-tiled, stage 1 LDS-tiled, stage 2
 * register-tiled, stage 2 LDS-tiled, stage 1 register-tiled narrow, stage 2 register-tiled
 * narrow, stage 1 LDS-staged, stage 2 LDS-staged, stage 1 K-split, stage 2 K-split] (-1 where
 * not timed).
 * Waits for the handle's stream. */
int dmrg_autotune(dmrg_handle h, int32_t reps, double* out);

/* Persisted autotuner (host-side cache; the tuner itself is dmrg_autotune).  The choice of the
 * autotuner depends on the architecture, the arithmetic and the sizes of the block products,
 * so a JSON file at path (UTF-8, created when missing) remembers it per key, the key being the
 * architecture name of the current device (gcnArchName up to its first ':'), the handle's
 * arithmetic, the problem count, the connection-term count and the histogram of the
 * superblock blocks' system and environment sector dimensions in buckets of 16 (see
 * dmrg_tune_key).  On a hit whose variant the handle can run, the variant is applied with no
 * device work; otherwise dmrg_autotune(h, reps, ...) runs and its choice and timings are stored
 * under the key (an entry of the same key is replaced).  out: NULL or 10 doubles receiving the
 * timings as in dmrg_autotune (those stored with the entry on a hit); hit: NULL or receives 1
 * on a hit, else 0.  The file is replaced by renaming a complete temporary file
 * (path.tmp.<pid>.<n>), so concurrent readers see the old or the new file; concurrent writers may
 * drop each other's new entries, which are timed again on their next miss.  Returns DMRG_EIO
 * (with the reason in dmrg_last_error) when the file exists but cannot be read or is not a
 * cache of this format (it is then left untouched), or when it cannot be written (the tuned
 * variant is applied all the same); DMRG_EINVAL for a NULL path or reps < 1. */
int dmrg_autotune_cached(dmrg_handle h, const char* path, int32_t reps, double* out,
                         int32_t* hit);

/* Key of a problem in the tuning cache (host only: no device is needed or used): arch is the
 * architecture name to key on (e.g. "gfx950"), precision a dmrg_precision.  Writes the key and a
 * terminating NUL to buf when cap exceeds its length; *len (not NULL) receives the length
 * without the NUL.  buf may be NULL to query the length.  DMRG_EINVAL for an invalid problem
 * (reason in dmrg_last_error(NULL)) or when buf is too short (nothing written). */
int dmrg_tune_key(const dmrg_problem* problem, int32_t precision, const char* arch, char* buf,
                  int64_t cap, int64_t* len);

/* Direct access to a tuning cache file (host only).  lookup: *found (not NULL) receives 1 and
 * *variant (not NULL) the stored bits when key is present (ms: NULL or 10 doubles receiving the
 * stored timings), else *found = 0.  store: adds or replaces the entry of key (ms: NULL, stored
 * as -1, or 10 doubles).  DMRG_EIO as for dmrg_autotune_cached, with the reason in
 * dmrg_last_error(NULL); DMRG_EINVAL for NULL arguments or unknown variant bits. */
int dmrg_tune_cache_lookup(const char* path, const char* key, int32_t* variant, double* ms,
                           int32_t* found);
int dmrg_tune_cache_store(const char* path, const char* key, int32_t variant, const double* ms);

/* Changes the stream all later work of the handle is ordered on. */
int dmrg_set_stream(dmrg_handle h, void* stream);

/* Input checking (off after dmrg_create).  When on, dmrg_matvec, dmrg_krylov_expm,
 * dmrg_tst_targets, dmrg_tst_chains, dmrg_ground_state and dmrg_batch_tst_targets first count
 * the NaN and infinite values of their input vectors on the device (one pass, then a wait for
 * the stream) and return DMRG_ENONFINITE without computing if there is any.  Without checking,
 * a Krylov call whose info is requested still returns DMRG_ENONFINITE when a step starts from a
 * vector with a non-finite norm (that step is then run as a zero vector). */
int dmrg_set_check_finite(dmrg_handle h, int32_t enable);

/* y = H_sb x for nvec vectors stored back to back (2n doubles each), device pointers.
 * x and y must not overlap.  Asynchronous on the handle's stream. */
int dmrg_matvec(dmrg_handle h, const double* x, double* y, int32_t nvec);

/* Bytes of device scratch per GPU held by the library for dmrg_matvec_noalloc. */
#define DMRG_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* dmrg_matvec for callers that cannot allocate device memory during the call: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Same arguments,
 * arithmetic and results (the same kernels and the same bits) as dmrg_matvec.  The call makes
 * no device allocation and no free: the stage-1 intermediate, which dmrg_matvec keeps in the
 * handle, lives here in a library-owned array of DMRG_NOALLOC_SCRATCH_BYTES on each GPU (held
 * from the library's load on that GPU until the process ends; its address is resolved by
 * dmrg_create).  Each call first clears the part it uses, with a kernel on the handle's stream.
 *   Every call on one GPU, from any handle, shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads) race and give wrong results; order them on one
 * stream.  The optional non-finite check (dmrg_set_check_finite) is not run.
 * Errors: DMRG_EINVAL for a null handle, negative nvec, null vectors with nvec > 0, or a
 * problem whose intermediate, in the layout of the handle's block-product family (the K-split
 * family pads it more), needs more than DMRG_NOALLOC_SCRATCH_BYTES (message via
 * dmrg_last_error; nothing is launched); DMRG_EHIP. */
int dmrg_matvec_noalloc(dmrg_handle h, const double* x, double* y, int32_t nvec);

/* y = (exp(-i tau H_sb))^nsteps x: nsteps Krylov steps of size kdim (1 <= kdim <= 64), each
 * from a fresh Lanczos basis of the current vector (Sec. II.A, Eq. lanczosevolution2).
 * x, y: device vectors; y may equal x.  If info is non-NULL the call waits for the stream
 * and fills it (and info->k_eff_steps, if set, with nsteps entries); otherwise it is
 * asynchronous.  DMRG_EINVAL for kdim outside [1, 64] or nsteps < 0; DMRG_ENONFINITE for a
 * non-finite tau, or as described at dmrg_set_check_finite. */
int dmrg_krylov_expm(dmrg_handle h, const double* x, double* y, double tau, int32_t kdim,
                     int32_t nsteps, dmrg_krylov_info* info);

/* Time-step targeting (Sec. II.B, II.C): from one Krylov basis of phi, the four vectors
 * phi(t_x) = exp(-i t_x H) phi at t_x = 0, tau/3, 2tau/3, tau, written to targets (device,
 * 4 x 2n doubles), and the five density-matrix weights [ground state, t_0, t_1, t_2, t_3] =
 * [2W, 2W, W, W, 2W], W = 1/8 (host array, may be NULL).  The next interval starts from
 * targets[3].  info as in dmrg_krylov_expm. */
int dmrg_tst_targets(dmrg_handle h, const double* phi, double tau, int32_t kdim,
                     double* targets, double* weights, dmrg_krylov_info* info);

/* Ground state of H_sb by restarted Lanczos (the ground-state target of Sec. II.B, weight 2W;
 * the same Krylov basis as dmrg_krylov_expm, Sec. II.A, with the lowest eigenpair of the
 * Lanczos matrix T in place of its exponential): up to max_restarts bases of kdim vectors, each
 * started from the previous Ritz vector (the first from x0), until the residual estimate
 * beta_kdim |z_{kdim-1}| = ||H y - E y|| is at most tol max(1, |E|).  y: the unit Ritz vector
 * (device, 2n doubles; may equal x0).  energy, restarts: NULL or host scalars receiving E and the
 * bases used; info as in dmrg_krylov_expm (err_est is the last residual estimate).  The call
 * waits for the stream after every basis (to test convergence).  Returns DMRG_WNOTCONV (with y,
 * energy and info of the last basis, info->converged = 0) when max_restarts bases end above
 * tol.  DMRG_EINVAL for kdim outside [1, 64], max_restarts < 1 or a negative tol. */
int dmrg_ground_state(dmrg_handle h, const double* x0, double* y, int32_t kdim,
                      int32_t max_restarts, double tol, double* energy, int32_t* restarts,
                      dmrg_krylov_info* info);

/* Reduced density matrix of the targets and its truncation (Sec. II.B): with every target in
 * the handle's sector, rho is block diagonal over the system sectors p,
 *   rho_p = sum_l weights[l] Psi_{l,p} Psi_{l,p}^H      (Psi_{l,p}: block p of vecs[l]),
 * and the keep eigenvectors with the largest eigenvalues over all sectors are kept (equal values
 * ranked by sector, then by position).  vecs: host array of nvec (1..16) device vectors;
 * weights: host array of nvec (the TST weights of dmrg_tst_targets for the ground state and the
 * four targets).  Outputs, per system sector in the order of dmrg_psi_layout (d = rows there):
 *   evals   device, sum of d doubles: eigenvalues of rho_p in descending order;
 *   evecs   device, sum of 2 d^2 doubles: per sector the d x d eigenvector matrix, column-major,
 *           real parts then imaginary parts, columns in the order of evals;
 *   kept    host int32 per sector: how many of its leading eigenvectors are kept;
 *   trunc_err  host (may be NULL): the sum of the discarded eigenvalues.
 * The eigen-decomposition per sector is Householder tridiagonalisation, bisection for the
 * eigenvalues, inverse iteration for the eigenvectors (implicit QL when close eigenvalues form a
 * cluster larger than 8) and back-transformation.  The call waits for the stream.  DMRG_EINVAL
 * for NULL arguments, nvec outside [1, 16], keep < 0 or a system sector larger than 1024 states;
 * DMRG_ENONFINITE for a weight that is not finite or a QL iteration that does not converge (64
 * sweeps per eigenvalue). */
int dmrg_density_truncate(dmrg_handle h, const double* const* vecs, const double* weights,
                          int32_t nvec, int32_t keep, double* evals, double* evecs, int32_t* kept,
                          double* trunc_err);

/* Wave-function transformation for a move of the centre one site to the right (Sec. II.B: the
 * targets are carried to the new superblock basis when the central sites change).  The
 * handle's superblock is (A x s1) x (s2 x R); the new one is S' x E' = (A' x s2) x (s3 x R''),
 * A' the kept states of each system sector (the first kept[b] eigenvectors of its density
 * matrix), R expressed in s3 x R'' by one matrix W_r per sector r of R:
 *   psi'[(alpha', a), gamma] = sum_{alpha, beta} conj(U[alpha, alpha']) psi[alpha, (a, beta)] W_r[gamma, beta].
 * The move is described by sector tables (all host arrays, copied by dmrg_wft_create):
 *   esub      [n_esub][4]: per sub-block of E = s2 x R: E sector q, site state a of s2 (0..3),
 *             R sector r, first column of the sub-block in sector q (its width is r_dim[r]);
 *   r_dim     [nr]: states of R sector r;  r_to_enew [nr]: the E' sector with r's quantum numbers;
 *   kept      [psi blocks of the handle, dmrg_psi_layout order]: states kept of that system
 *             sector (0 drops it; at most its d);
 *   ssub      [n_ssub][4]: per sub-block of S' = A' x s2: psi block b, site state a, S' sector,
 *             first row of the sub-block in it (its height is kept[b]);
 *   s_new_qn  [ns_new][2], s_new_dim [ns_new]: sectors of S' (sorted, distinct);
 *   e_new_qn  [ne_new][2], e_new_dim [ne_new]: sectors of E' (sorted, distinct).
 * The new vector has the handle's target sector and the layout dmrg_psi_layout would give S'
 * and E' (blocks in S' sector order, column-major, real parts then imaginary parts). */
typedef struct {
    int32_t n_esub;
    const int32_t* esub;
    int32_t nr;
    const int32_t* r_dim;
    const int32_t* r_to_enew;
    const int32_t* kept;
    int32_t n_ssub;
    const int32_t* ssub;
    int32_t ns_new;
    const int32_t* s_new_qn;
    const int32_t* s_new_dim;
    int32_t ne_new;
    const int32_t* e_new_qn;
    const int32_t* e_new_dim;
} dmrg_wft_desc;

typedef struct dmrg_wft_ctx* dmrg_wft;

/* Plans a move for handle h.  W: host array of nr device pointers, W[r] holding the complex
 * d_E'(r_to_enew[r]) x r_dim[r] matrix W_r, column-major, real parts then imaginary parts; the
 * matrices are copied (the caller may free them after the call).  n_new (may be NULL): complex
 * length of the new vector.  DMRG_EINVAL for a description that is out of range or
 * inconsistent (a sub-block outside its sector, quantum numbers that do not add up to the
 * target, S' rows covered twice). */
int dmrg_wft_create(dmrg_handle h, const dmrg_wft_desc* desc, const double* const* W, dmrg_wft* out,
                    int64_t* n_new);

/* Transforms nvec (1..16) vectors: x[v] (device, 2n doubles of the handle's layout) to y[v]
 * (device, 2 n_new doubles; must not overlap x).  U: device, the eigenvector array written by
 * dmrg_density_truncate for the handle (per sector, d x d, real then imaginary planes).  The
 * intermediate is allocated on first use for the largest nvec seen.  Asynchronous on the
 * handle's stream.  flops (may be NULL): algorithmic flops of the call. */
int dmrg_wft_apply(dmrg_wft w, const double* U, int32_t nvec, const double* const* x,
                   double* const* y, double* flops);

/* Releases a planned move (waits for the handle's stream).  Destroy every move of a handle
 * before the handle.  DMRG_EINVAL for NULL. */
int dmrg_wft_destroy(dmrg_wft w);

/* Local operators on the superblock (Sec. II.B, Eq. (b): the operators B applied to the ground
 * state to form phi; Sec. III.B: the measured densities n_p and double occupations): with the
 * same halves in both handles,
 *   y = sum_t terms[t].coef (A_t P_S^f_t (x) B_t) x,
 * A_t = src's S.ops[opS] (transposed if transS; opS = -1: the identity), B_t = src's E.ops[opE]
 * likewise, P_S the fermion parity of the system (f_t = terms[t].fermionic: set it when B_t is
 * odd, since B_t then passes the system's modes).  x: device, src's layout; y: device, dst's
 * layout (dst's target = src's target plus the quantum numbers the terms add); y is
 * overwritten and must not be x.  Operator blocks of src that have no image in dst's sector
 * contribute nothing.  Asynchronous on src's stream.  DMRG_EINVAL for different halves, an
 * operator index out of range or a term that does not map src's target to dst's. */
int dmrg_apply_local(dmrg_handle src, dmrg_handle dst, int32_t nterm, const dmrg_term* terms,
                     const double* x, double* y);

/* <x| sum_t terms[t] |x> for terms that keep the handle's sector (as in dmrg_apply_local with
 * src = dst = h): re, im (host, may be NULL) receive its real and imaginary parts.  Fixed-order
 * reduction; the call waits for the stream. */
int dmrg_expect_local(dmrg_handle h, int32_t nterm, const dmrg_term* terms, const double* x,
                      double* re, double* im);

/* 4-RHS (per-target) mode of time-step targeting: the four targets are kept as four independent
 * chains, each advanced by exp(-i tau H) with a Krylov basis of its own (kdim vectors, Sec. II.A)
 * instead of one basis evaluated at four times (the variant of the seeding of the next
 * interval, Sec. II.C; it agrees with dmrg_tst_targets only to Krylov error).  The four chains
 * share every block-product and vector-pass launch; in FP64 with narrow tiles in both stages
 * (DMRG_GEMM_STAGE1_NARROW | DMRG_GEMM_STAGE2_NARROW) one stage-2 work group computes a tile
 * for all four chains, loading the packed left factors once.  Each target has the same bits as
 * one dmrg_krylov_expm step of its phi with the same kdim.  phi, targets: host arrays of 4 device
 * pointers (2n doubles each); targets[k] = exp(-i tau H) phi[k], and targets[k] may equal
 * phi[k].  weights as in dmrg_tst_targets.  infos: NULL or a host array of 4 structs (then the
 * call waits for the stream).  The first call allocates three more workspaces of the handle's
 * size (intermediate, basis, vectors). */
int dmrg_tst_chains(dmrg_handle h, const double* const* phi, double tau, int32_t kdim,
                    double* const* targets, double* weights, dmrg_krylov_info* infos);

/* Runs the kdim Lanczos iterations of dmrg_krylov_expm and dmrg_tst_targets as one HIP graph
 * (captured on first use per kdim on a private stream, launched on the handle's stream;
 * re-captured after the workspace or the precision changes) instead of one launch per pass.
 * Off by default.  Results are identical either way. */
int dmrg_set_graph(dmrg_handle h, int32_t enable);

/* Batched time-step targeting over independent superblocks (Sec. II.B applied to many
 * superblocks at once; handles created beforehand, distinct, all set to one precision).  The
 * batch merges the block-product work lists of all handles into one launch per stage and runs
 * every Lanczos pass for all of them in one launch; the kdim iterations run as one HIP graph
 * unless dmrg_batch_set_graph(b, 0).  The batch keeps references: the handles must outlive it
 * and must not be used concurrently with it.  Its work is ordered on the stream of the first
 * handle; errors of batch calls are described by dmrg_last_error of the first handle. */
int dmrg_batch_create(const dmrg_handle* handles, int32_t count, dmrg_batch* out);
void dmrg_batch_destroy(dmrg_batch b);
int dmrg_batch_set_graph(dmrg_batch b, int32_t enable);

/* Kernel families of the batch's merged launches (initially those of the first handle), and
 * their autotuner (as dmrg_autotune, on the merged work lists of all handles). */
int dmrg_batch_set_gemm(dmrg_batch b, int32_t variant);
int dmrg_batch_autotune(dmrg_batch b, int32_t reps, double* out);
/* As dmrg_autotune_cached, for the batch's merged launches: the key counts the problems, terms
 * and blocks of all member handles in the arithmetic of the batch's tables. */
int dmrg_batch_autotune_cached(dmrg_batch b, const char* path, int32_t reps, double* out,
                               int32_t* hit);

/* phi[i], targets[i]: device pointers for superblock i (host arrays of count pointers; the
 * targets of superblock i are 4 x 2 n_i doubles).  Results equal those of dmrg_tst_targets on
 * each handle.  weights as in dmrg_tst_targets.  infos: NULL or a host array of count structs
 * (then the call waits for the stream).  DMRG_EINVAL if a pointer is NULL or the handles use
 * different precisions. */
int dmrg_batch_tst_targets(dmrg_batch b, const double* const* phi, double tau, int32_t kdim,
                           double* const* targets, double* weights, dmrg_krylov_info* infos);

/* The 4-RHS mode for every superblock of the batch in common launches: phi, targets: host
 * arrays of 4 x count device pointers, chain k of superblock i at [4 i + k].  Results equal those
 * of dmrg_tst_chains on each handle.  infos: NULL or 4 x count structs. */
int dmrg_batch_tst_chains(dmrg_batch b, const double* const* phi, double tau, int32_t kdim,
                          double* const* targets, double* weights, dmrg_krylov_info* infos);

/* Measurement hook: one product y = H_sb x (one vector), then reps launches of the right-product
 * stage back to back and reps launches of the left-product stage back to back, with HIP events
 * on the handle's stream around each run; waits for them.  out[0], out[1]: average
 * milliseconds per launch of the two stages; out[2], out[3]: the flops each stage executes
 * (their sum is dmrg_flops_executed).  y holds H_sb x afterwards. */
int dmrg_profile_matvec(dmrg_handle h, const double* x, double* y, int32_t reps, double* out);

/* Static description of a status code. */
const char* dmrg_strerror(int status);

/* Description of the last error on a handle (empty string if none; never NULL).  With
 * h = NULL: the reason the calling thread's last dmrg_create() failed. */
const char* dmrg_last_error(dmrg_handle h);

#ifdef __cplusplus
}
#endif

#endif /* DMRGTST_H */

/*
 * libgmres: restarted GMRES(m) for sparse non-symmetric systems on gfx950.
 *
 * Method: Lindquist, Luszczek, Dongarra, "Improving the Performance of the
 * GMRES Method using Mixed-Precision Techniques" (arXiv 2011.01850).
 * Algorithm 1 (restarted GMRES, MGS or CGSR orthogonalisation) runs with the
 * precision split of the paper's numerics section: the restart residual
 * z = b - A x and the update x += u are float64, the Arnoldi process
 * (SpMV, orthogonalisation, normalisation) runs in float32, or stores its
 * basis in bfloat16 / IEEE half with a per-vector power-of-two scale.  The
 * Hessenberg matrix, its Givens rotations and the back-solve are float64.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers unless stated otherwise
 *    (e.g. torch tensors on the current HIP device).  Options and results
 *    are host structs.
 *  - CSR: row_ptr int32[n+1] (row_ptr[0] = 0, non-decreasing), col_idx
 *    int32[nnz] in [0, n), values float64[nnz].  Column order inside a row
 *    is free and duplicates are summed, except with GMRES_PRECOND_ILU0
 *    (increasing columns, see below).
 *  - Return value: GMRES_OK (0) or a negative error code (gmres_strerror).
 *    Not converging is not an error: gmres_solve returns GMRES_OK and
 *    reports the outcome in gmres_result.status.
 *  - Every handle owns a non-blocking stream of default priority on which
 *    all its device work runs.  Each call that reads or writes caller memory
 *    first makes that stream wait for the work already enqueued on the
 *    caller's stream (the hip_stream given at creation; NULL = the null
 *    stream), and returns only after its own stream has drained, so caller
 *    memory may be used on the caller's stream as soon as the call returns.
 *    A handle must be used by one host thread at a time.
 */
#ifndef GMRES_H_
#define GMRES_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmres_ctx* gmres_handle;

/* orthogonalisation of Algorithm 1: modified Gram-Schmidt, or classical
 * Gram-Schmidt with one full re-orthogonalisation pass (two projections,
 * coefficients summed). */
enum { GMRES_MGS = 0, GMRES_CGSR = 1 };

/* precision of the Arnoldi process (numerics section; 2-byte formats follow
 * the half-precision direction of the conclusion).  The residual, the update,
 * H, the rotations and the back-solve are float64 in every mode. */
enum {
  GMRES_FP64 = 0,       /* everything float64 (the baseline) */
  GMRES_MIXED_FP32 = 1, /* float32 A copy, basis, w and dot products */
  GMRES_MIXED_BF16 = 2, /* float32 arithmetic, basis stored as bfloat16 */
  GMRES_MIXED_FP16 = 3, /* float32 arithmetic, basis stored as IEEE half */
  /* the limited mixed solver of the convergence study (section 4.1): only
   * the storage of A for the Arnoldi product, of the preconditioner and of
   * the basis is float32; w, its dot products and the Arnoldi product's
   * sums are float64 (float32 values widened exactly).  Basis traffic as in
   * GMRES_MIXED_FP32, w traffic as in GMRES_FP64.  Not available with the
   * persistent batch schedule. */
  GMRES_MIXED_LIMITED = 4
};

/* gmres_options.a_storage: how the handle keeps A's values.
 * COPY:  the float64 values plus a float32 copy for the Arnoldi SpMV
 *        (12 bytes per non-zero in the mixed modes, as in the numerics
 *        section of the paper, which notes that the matrix is stored twice).
 * SPLIT: the float64 values split into two arrays of 32-bit words, high
 *        words and low words (8 bytes per non-zero; the storage the paper
 *        suggests as an improvement, after the modular-precision format it
 *        cites).  The float64 residual SpMV reads both; the Arnoldi SpMV of
 *        the mixed modes reads the high words only, i.e. each value truncated
 *        to 20 significand bits (relative error below 2^-20), converted
 *        exactly to float32.  Not available with the persistent batch
 *        schedule. */
enum { GMRES_A_COPY = 0, GMRES_A_SPLIT = 1 };

/* right preconditioning in flexible GMRES (z_j = M v_j, w = A z_j, x += Z y).
 * ILU0: incomplete LU without fill (the preconditioner of the paper's
 * experiments), factored on the GPU in float64 at create time (rows in
 * dependency levels; every row must store its diagonal and list its columns
 * in increasing order, else gmres_create returns GMRES_EINVAL) and applied as
 * z = U^-1 L^-1 v by ilu_sweeps Jacobi sweeps per triangle from a zero
 * start, or exactly (ilu_sweeps = 0: as many sweeps as the triangle has
 * levels).  The paper applies ILU(0) on the left; here it is applied on the
 * right, so GMRES keeps minimising the true residual.
 * Precision (Algorithm 1's M^-1 and the paper's split of Section 4.2): the
 * mixed modes store and apply the preconditioner in float32 and keep Z in
 * float32.  GMRES_FP64 keeps Z in float64 and applies the preconditioner in
 * float64 (Jacobi d^-1, the ILU factors and sweeps), or, with
 * precond_precision = GMRES_PRECOND_FP32, in float32 (the paper's "FP32
 * ILU only" solver: v_j rounded to float32, float32 factors and sweeps, the
 * result widened to float64).  The learned M (float32 values) is summed in
 * the precision of Z. */
enum { GMRES_PRECOND_NONE = 0, GMRES_PRECOND_JACOBI = 1, GMRES_PRECOND_SPAI = 2, GMRES_PRECOND_ILU0 = 3 };

/* gmres_options.batch_schedule.
 * DEVICE_WIDE: every kernel launch covers all systems of the handle (any
 * options); one restart cycle is one graph launch.
 * PERSISTENT: one kernel launch for the whole solve; each workgroup of 1024
 * threads takes systems from a queue (largest first) and runs Algorithm 1
 * on one system with its work vector in registers.  Requires MIXED_FP32,
 * MGS, no preconditioner, m <= 64 and n <= 65536 for every system.
 * AUTO: PERSISTENT for batch handles (gmres_batch_create) that meet those
 * conditions, DEVICE_WIDE otherwise. */
enum { GMRES_SCHEDULE_AUTO = 0, GMRES_SCHEDULE_DEVICE_WIDE = 1, GMRES_SCHEDULE_PERSISTENT = 2 };

/* gmres_result.status.  Breakdown of the Arnoldi process (h_{j+1,j} = 0 in
 * Algorithm 1, detected here as h_{j+1,j} <= 16 (j+1) u ||A v_j|| with u the
 * unit roundoff of the Arnoldi arithmetic) has no status of its own: it ends
 * the cycle like j = m does, the correction from the columns formed so far
 * is applied, and the float64 restart residual decides what follows.  A
 * "lucky" breakdown (the Krylov space holds the solution) therefore ends as
 * CONVERGED.  A breakdown whose least-squares problem keeps no column (every
 * leading pivot of H below 16 k u max|H|, e.g. A v_1 = 0 for a singular A)
 * applies no correction, so the restart residual does not move and the solve
 * ends as STALLED after stall_cycles such cycles. */
enum { GMRES_RUNNING = 0, GMRES_CONVERGED = 1, GMRES_MAXITER = 2, GMRES_STALLED = 3 };

/* error codes */
enum {
  GMRES_OK = 0,
  GMRES_EINVAL = -1,  /* invalid argument: n <= 0, m < 1 or m > 256, tol < 0, bad CSR, NULL pointer,
                         or sizes the kernels cannot address (checked before any device work):
                         padded rows (each system's n rounded up to a multiple of 256, summed)
                         >= 2^31 - 1, non-zeros > 2^31 - 1029, or a basis of (m + 1) x padded
                         rows x element bytes (8 float64, 4 float32 / limited, 2 bfloat16 / half)
                         >= 2^32 bytes, since the basis is read through 32-bit buffer offsets */
  GMRES_EHIP = -2,    /* a HIP runtime call failed */
  GMRES_ENOMEM = -3,  /* device allocation failed */
  GMRES_EHANDLE = -4, /* NULL or destroyed handle */
  GMRES_ESTATE = -5   /* call not valid for this handle (e.g. SPAI values on a handle created without SPAI) */
};

typedef struct {
  int32_t m;                /* restart length, 1..256 */
  double tol;               /* stop when ||b - A x||_2 / ||b||_2 <= tol (float64 residual) */
  int64_t max_iters;        /* budget of inner (Arnoldi) iterations over all cycles */
  int32_t ortho;            /* GMRES_MGS or GMRES_CGSR */
  int32_t precision;        /* GMRES_FP64 ... GMRES_MIXED_LIMITED */
  int32_t precond;          /* GMRES_PRECOND_* */
  double restart_improve;   /* 0 = off; else end a cycle once |s_{j+1}| <= restart_improve * beta
                               (the improvement trigger of the restart-strategy study) */
  int32_t stall_cycles;     /* STALLED after this many cycles in a row that do not lower the best
                               restart residual so far (a 2-byte basis makes single cycles noisy) */
  int32_t use_graph;        /* 1: capture one restart cycle as a hipGraph and replay it */
  int32_t autotune;         /* 1: time SpMV tile variants at create time and keep the fastest */
  int32_t batch_schedule;   /* GMRES_SCHEDULE_*: how the systems of a handle share the GPU */
  int32_t spmv_block_nnz;   /* 0: SpMV row blocks chosen by the autotuner (autotune = 1) or 2048;
                               else a fixed non-zero budget per row block, a multiple of 64 in
                               [64, 8192]; a block holds up to 256 rows (512 with budgets of 4096
                               and more).  Results do not depend on it: every row is summed in
                               one order fixed by its length. */
  int32_t a_storage;        /* GMRES_A_COPY or GMRES_A_SPLIT */
  /* Restart strategies of the restart study (section 3), each optional and
   * combinable with j = m and the improvement trigger above:
   * restart_repeat   1: the first cycle ends as usual (m, or restart_improve);
   *                  every later cycle ends after as many inner iterations as
   *                  the first one took (the two-stage strategy; the
   *                  improvement trigger applies to the first cycle only).
   * restart_on_stall 1: end a cycle once the Arnoldi residual stalls, i.e.
   *                  |s_{j+1}| > |s_{j+1-w}| / 1.001 with w = max(1, ceil(0.05 m))
   *                  (the third strategy; the same window as first_stall).
   * orth_restart     > 0: end a cycle once ||S_k|| >= orth_restart, where
   *                  S_k = (I + U_k)^-1 U_k and U_k is the strictly upper part
   *                  of V_k^T V_k (the loss-of-orthogonality strategy; ||S_k|| = 1
   *                  exactly when the basis is linearly dependent).  Costs one
   *                  more pass over the basis per step.
   * orth_norm        GMRES_ORTH_SPECTRAL (10 power iterations on S_k^T S_k from
   *                  the all-ones vector) or GMRES_ORTH_FROBENIUS. */
  int32_t restart_repeat;
  int32_t restart_on_stall;
  double orth_restart;
  int32_t orth_norm;
  int32_t ilu_sweeps;       /* GMRES_PRECOND_ILU0: Jacobi sweeps per triangle (0 = exact), 0..4096 */
  int32_t arnoldi_a;        /* GMRES_ARNOLDI_A_*: which values of A the Arnoldi product reads */
  int32_t precond_precision; /* GMRES_PRECOND_NATIVE (the solver's precision) or GMRES_PRECOND_FP32
                                (a float32 preconditioner in the float64 solver) */
  int32_t persistent_spmv;   /* persistent batch schedule: 0 = the Arnoldi SpMV variant chosen by the
                                create-time tuner (autotune = 1; else CSR8); 1 + GMRES_PSPMV_* forces
                                one */
  int32_t precond_side;      /* GMRES_PRECOND_RIGHT (flexible GMRES, the default) or GMRES_PRECOND_LEFT */
  int32_t spmv_format;       /* GMRES_SPMV_*: the Arnoldi product's layout (device-wide schedule) */
} gmres_options;

/* gmres_options.spmv_format.  CSR: the adaptive row blocks (spmv_block_nnz).
 * SELL: a sliced ELL copy of the values the Arnoldi product reads (64-row
 * slices, entry k of a slice's rows contiguous, so each load of a wave is
 * coalesced; 4 bytes of column and 4 or 8 of value per entry, padded to the
 * slice's longest row, plus a byte of length per row), built at create; only
 * when every row has fewer than 8 entries (then each row's sum is the plain
 * sum in storage order, so both layouts give the same bits) and split storage
 * is off, else CSR.  SELL16: the same copy with each column stored as a
 * 16-bit offset from its row (2 bytes instead of 4) when every column of the
 * matrix is within 32767 of its row, else as SELL.  AUTO: the sliced copy
 * (16-bit offsets when they fit) competes with the row-block budgets in the
 * autotuner (autotune = 1), else CSR.  All layouts give the same bits.  The
 * residual and preconditioner products always use the row blocks. */
enum { GMRES_SPMV_AUTO = 0, GMRES_SPMV_CSR = 1, GMRES_SPMV_SELL = 2, GMRES_SPMV_SELL16 = 3 };

/* gmres_options.precond_side.  RIGHT: flexible GMRES, z_j = M^-1 v_j kept,
 * w = A z_j, x += Z y.  LEFT, the form of the paper's experiments
 * (Algorithm 1 with M^-1 on the left): each cycle starts from
 * r = M^-1 (b - A x) (the residual in float64, M^-1 applied in the
 * preconditioner's precision to w's copy of it), beta = ||r||, and every
 * step forms w = M^-1 A v_j; x += V y.  The inner loop compares its estimate
 * |s_{j+1}| (of ||M^-1 (b - A x)||) with tol ||M^-1 b||; the float64
 * restart residual ||b - A x|| / ||b|| stays the stop test.  A zero or
 * non-finite M^-1 z switches the preconditioner off (fallback_used), as a
 * cycle that gains less than 1.001x does on either side. */
enum { GMRES_PRECOND_RIGHT = 0, GMRES_PRECOND_LEFT = 1 };

/* Arnoldi SpMV variants of the persistent batch kernel (all sum each row's
 * products in storage order, so the choice never changes a result bit):
 * CSR8 / CSR4: the CSR arrays, a row's entries loaded in groups of 8 / 4;
 * ELL16: an ELL copy made at create (entry k of every row of a system in one
 * contiguous slice, 16-bit columns local to the system, a byte of row
 * length; only when every system of the batch has at most 65,536 rows with
 * at most 255 entries each, else CSR8 runs instead).  One variant runs for
 * the whole batch (one persistent kernel per variant). */
enum { GMRES_PSPMV_CSR8 = 0, GMRES_PSPMV_CSR4 = 1, GMRES_PSPMV_ELL16 = 2 };

enum { GMRES_PRECOND_NATIVE = 0, GMRES_PRECOND_FP32 = 1 };

enum { GMRES_ORTH_SPECTRAL = 0, GMRES_ORTH_FROBENIUS = 1 };

/* gmres_options.arnoldi_a, for the per-variable study of section 4.1 (one
 * variable of the correction in single precision, the rest unchanged):
 * DEFAULT  float64 values with GMRES_FP64, float32 values (the float32 copy,
 *          or the high words under SPLIT storage) in every mixed mode.
 * FP64     the float64 values in any mode (no float32 copy is kept); with
 *          GMRES_MIXED_LIMITED this leaves the basis (and M) as the only
 *          float32 variables.
 * FP32     the float32 values in any mode; with GMRES_FP64 this makes A for
 *          the next Krylov vector the only float32 variable.
 * The product's sums are float64 whenever w or the values are float64.
 * FP32 is the only choice with the persistent batch schedule. */
enum { GMRES_ARNOLDI_A_DEFAULT = 0, GMRES_ARNOLDI_A_FP64 = 1, GMRES_ARNOLDI_A_FP32 = 2 };

typedef struct {
  int32_t status;        /* GMRES_CONVERGED / MAXITER / STALLED */
  int64_t iters;         /* inner Arnoldi iterations, summed over cycles */
  int64_t restarts;      /* completed cycles (corrections applied) */
  double rel_residual;   /* ||b - A x||_2 / ||b||_2 in float64, at exit */
  double seconds;        /* wall time of the solve call (setup excluded) */
  int32_t fallback_used; /* the preconditioner was switched off (stall or non-finite values) */
  int32_t first_stall;   /* inner iterations before the Arnoldi residual stalled in the first
                            cycle (improvement < 1.001x over the next 5% of m); -1 if none */
} gmres_result;

/* Fill *opt with defaults: m = 50, tol = 1e-10, max_iters = 100000, CGSR,
 * MIXED_FP32, no preconditioner, restart_improve = 0, stall_cycles = 10,
 * use_graph = 1, autotune = 1, batch_schedule = AUTO, spmv_block_nnz = 0, a_storage = COPY,
 * restart_repeat = 0, restart_on_stall = 0, orth_restart = 0, orth_norm = SPECTRAL, ilu_sweeps = 4,
 * arnoldi_a = DEFAULT, precond_precision = NATIVE, persistent_spmv = 0, precond_side = RIGHT,
 * spmv_format = AUTO. */
void gmres_default_options(gmres_options* opt);

/* Create a solver for one n x n system (Algorithm 1, inputs A, M^-1).
 * Copies A into library storage (float64 values, a float32 copy for the
 * mixed modes, shared indices, SpMV row blocks), allocates the workspace
 * (basis of m+1 vectors, H, rotations, reductions) and, if requested, runs
 * the SpMV autotuner.  The caller may free its CSR arrays afterwards.
 * hip_stream: the caller's hipStream_t (NULL = the null stream) that the
 * handle's calls are ordered after; it is not used for the library's work.
 * Errors: EINVAL (n <= 0, nnz < 0, NULL pointers, bad options, bad CSR),
 * ENOMEM, EHIP. */
int gmres_create(gmres_handle* out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col_idx, const double* vals, const gmres_options* opt,
                 void* hip_stream);

/* Create one solver for nsys independent systems (the batch path): the
 * k-th system is n[k] x n[k] with nnz[k] entries given by the k-th pointers
 * of the (HOST) pointer arrays, which point to device memory.  Each system
 * keeps its own Hessenberg matrix, rotations, restart and stop decisions.
 * Under the device-wide schedule its iterates are exactly those of a
 * single-system solve; under the persistent schedule, exactly those of a
 * persistent solve of that system alone.  Errors as gmres_create, and
 * EINVAL for batch_schedule = PERSISTENT when its conditions fail. */
int gmres_batch_create(gmres_handle* out, int32_t nsys, const int64_t* n, const int64_t* nnz,
                       const int32_t* const* row_ptr, const int32_t* const* col_idx,
                       const double* const* vals, const gmres_options* opt, void* hip_stream);

/* The preconditioner M^-1 of Algorithm 1's inputs, given explicitly:
 * values of a sparse approximate inverse M on the sparsity pattern of A
 * (float32, device, one value per stored entry of A in A's storage order,
 * systems concatenated for a batch handle).  Used as z = M v in the
 * flexible (right-preconditioned) solve.  Errors: ESTATE unless the handle
 * was created with precond = GMRES_PRECOND_SPAI. */
int gmres_set_preconditioner(gmres_handle h, const float* spai_vals);

/* Solve A x = b by Algorithm 1: restart cycles of float64 residual
 * z = b - A x and stop test, m Arnoldi steps (SpMV, MGS or CGSR, Givens
 * update of H), back-solve and float64 correction x += V y (x += Z y in the
 * flexible form), with the precision split of the numerics section.
 * b: float64[n], read only.  x: float64[n], in: x0, out: the final iterate.
 * b = 0 gives x = 0 with 0 iterations.  Synchronises the stream and fills
 * *res (res may be NULL). */
int gmres_solve(gmres_handle h, const double* b, double* x, gmres_result* res);

/* Batch solve: b[k], x[k] are device pointers of system k (host arrays of
 * nsys pointers); res is a host array of nsys results. */
int gmres_batch_solve(gmres_handle h, const double* const* b, double* const* x, gmres_result* res);

/* Free everything owned by the handle.  Safe on NULL.  Waits for the
 * handle's stream; its device blocks are kept by the library for the next
 * handle created on the same device (up to 16 GiB per device; beyond that,
 * and for any block when a new allocation fails, they are freed). */
int gmres_destroy(gmres_handle h);

/* Frees the device blocks destroyed handles left for reuse, on every device
 * (live handles keep theirs); *bytes (HOST, may be NULL) = the bytes freed.
 * Not to be called while another thread creates a handle. */
int gmres_release_cached_memory(size_t* bytes);

const char* gmres_strerror(int code);

/* r = b - A x in float64 with the stored A, and *norm_out = ||r||_2 (host,
 * may be NULL).  r may be NULL when only the norm is wanted.  b, x, r:
 * float64[n] device.  Single-system handles only (ESTATE on a batch handle). */
int gmres_residual(gmres_handle h, const double* b, const double* x, double* r, double* norm_out);

/* The stopping metric of the paper's experiments (Section 4.2): the
 * normwise backward error eta = ||b - A x||_2 / (||A|| ||x||_2 + ||b||_2),
 * with the Frobenius norm ||A||_F standing in for ||A||_2 (which it bounds
 * from above, so eta is at most sqrt(n) times too small), all in float64
 * with the stored A.  *eta and *rel_residual (= ||b - A x||_2 / ||b||_2)
 * are host outputs, either may be NULL.  b, x: float64[n] device.
 * Single-system handles only (ESTATE on a batch handle). */
int gmres_backward_error(gmres_handle h, const double* b, const double* x, double* eta, double* rel_residual);

/* The unit restart residual of Algorithm 1 in float32: r_out = float32(z /
 * ||z||_2) with z = b - A x computed in float64 (the first basis vector of
 * a cycle before its storage format is applied), and *norm_out = ||z||_2
 * (host, may be NULL).  Used to collect the residuals the learned
 * preconditioner trains on.  b, x: float64[n] device; r_out: float32[n]
 * device.  EINVAL when ||z|| is 0 or not finite (r_out untouched).
 * Single-system handles only. */
int gmres_residual_unit(gmres_handle h, const double* b, const double* x, float* r_out, double* norm_out);

/* y = A x with the stored float64 values (precision = GMRES_FP64, x and y
 * float64) or the float32 values of the Arnoldi product (GMRES_MIXED_FP32,
 * float32 x, y: the float32 copy, or the high words under SPLIT storage;
 * GMRES_MIXED_LIMITED: the same values and float32 x, summed in float64,
 * float64 y).  The float32 values exist only on mixed-precision handles
 * (else ESTATE); single-system handles only (ESTATE on a batch handle). */
int gmres_spmv(gmres_handle h, int32_t precision, const void* x, void* y);

/* z = M^-1 v for a single-system handle created with
 * precond = GMRES_PRECOND_ILU0: the ILU(0) application of the Arnoldi loop
 * (sweeps as configured by ilu_sweeps).  gmres_precond_apply: v and z are
 * float32[n] device arrays, for handles whose preconditioner computes in
 * float32 (the mixed modes; GMRES_FP64 with GMRES_PRECOND_FP32, whose z is
 * then float32 before widening).  gmres_precond_apply_f64: float64[n], for
 * GMRES_FP64 handles with a float64 preconditioner.  Errors: EINVAL (null
 * pointer), ESTATE (another preconditioner, the other precision, or
 * several systems). */
int gmres_precond_apply(gmres_handle h, const float* v, float* z);
int gmres_precond_apply_f64(gmres_handle h, const double* v, double* z);

/* Store v = w * inv_h in a 2-byte format (precision GMRES_MIXED_BF16 or
 * GMRES_MIXED_FP16) exactly as the solver stores a basis vector: with
 * e such that max|v| * 2^e lies in (T/2, T] (T = 1 for bfloat16, 2^15 for
 * half), out = round_to_nearest_even(float32(w * float32(2^e * inv_h))), and
 * *scale_out = 2^-e (host) so that v ~ out * scale.  w: float32[n] device;
 * out: uint16[n] device.  Runs on hip_stream and synchronises it. */
int gmres_encode(int32_t precision, int64_t n, const float* w, double inv_h, void* out,
                 double* scale_out, void* hip_stream);

/* gmres_encode without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same arguments, result and scale as
 * gmres_encode, bit for bit.  The per-tile partial maxima live in a static
 * device array of 262,400 bytes (one float per 256-element tile of at most
 * 2^24 elements, plus the reduced maximum) that each GPU the library runs on
 * holds until the process ends.  n > 2^24 is refused with GMRES_EINVAL
 * before any device work.  Every call on one GPU uses that GPU's array, so
 * calls that overlap in time on one GPU (other host threads, other streams)
 * race; calls in sequence do not (each call writes every slot it reads).
 * Runs on hip_stream and synchronises it. */
int gmres_encode_noalloc(int32_t precision, int64_t n, const float* w, double inv_h, void* out,
                         double* scale_out, void* hip_stream);

/* After a solve, the last cycle of system sys: *k_out = number of Arnoldi
 * steps, Hbar_out (HOST, float64, (m+1) x m column-major, may be NULL) =
 * the unrotated Hessenberg matrix, V_out (DEVICE, float64, n x (k+1)
 * column-major, may be NULL) = the decoded basis vectors (v_{k+1} only
 * when it was formed).  For tests of the Arnoldi relation. */
int gmres_last_cycle(gmres_handle h, int32_t sys, int32_t* k_out, double* Hbar_out, double* V_out);

/* Float64 relative restart residuals of system sys (HOST out[cap]); *count
 * = number recorded in the last solve (at most cap are copied). */
int gmres_history(gmres_handle h, int32_t sys, double* out, int32_t cap, int32_t* count);

/* Device bytes held by the handle (matrix copies, workspace, scratch). */
int gmres_memory_bytes(gmres_handle h, size_t* bytes);

/* Kernel timing harness for the roofline report: launches one hot-path
 * kernel `reps` times at Arnoldi column j with the solver's own launch
 * configuration, between HIP events on the handle's stream, and returns
 * the mean duration in milliseconds (*avg_ms) and the algorithmic bytes
 * one launch must move (*bytes).  The handle's solver state is clobbered
 * (the next gmres_solve starts afresh).  kernel: 0 = Arnoldi SpMV,
 * 1 = CGSR projection pass 1, 2 = CGSR projection pass 2, 3 = final
 * update + norm pass, 4 = MGS dot step (column j), 5 = float64 residual,
 * 6 = float64 solution update (j + 1 columns), 7 = the per-system reduction
 * that completes projection pass 2.  Kernels 1-5 are timed without their
 * completing reduction, which the solver launches right after them.  One
 * untimed launch precedes the timed ones; the timed launches run back to
 * back, so caches hold only what the previous launch of the same kernel
 * left (inside a solve, pass 2 follows pass 1 over the same columns).  The
 * timed launches sit inside a ROCTx range "timed:<kernel>" when the ROCTx
 * library can be loaded, for profilers that rename kernels by range. */
int gmres_time_kernel(gmres_handle h, int32_t kernel, int32_t j, int32_t reps, double* avg_ms,
                      double* bytes);
/* (ESTATE on a handle that runs the persistent batch schedule.) */

/* In-solve kernel profile (measurement of Algorithm 1's steps inside a real
 * solve).  gmres_solve_profiled runs the same solve as gmres_solve, the same
 * kernels in the same order with the same launch configurations (so x, the
 * iteration count and the history are bitwise those of gmres_solve), but
 * launches every kernel directly instead of through the per-cycle graph and
 * brackets each group of launches with a pair of HIP events on the handle's
 * stream.  prof (HOST, GMRES_PK_COUNT entries) receives per kernel family:
 * the summed event-timed durations of all its launches (ms, launches) and
 * of the launches that did work (ms_active, active: a step j >= k of a
 * cycle that ended after k steps is gated off on the device and returns at
 * once), and the algorithmic bytes the active launches move (the formulas
 * of the design notes: e.g. projection 1 at column j reads j+1 basis
 * columns and w).  Single-system handles on the device-wide schedule only
 * (ESTATE otherwise).  Families: */
enum {
  GMRES_PK_SPMV = 0,      /* Arnoldi product w = A v_j (or A z_j) */
  GMRES_PK_PASS1 = 1,     /* CGSR projection 1: V^T w */
  GMRES_PK_PASS2 = 2,     /* CGSR projection 2: w -= V h1, then V^T w */
  GMRES_PK_FINAL = 3,     /* last pass of a step: w -= V h2 (CGSR) or the last MGS axpy; ||w||, v_{j+1} */
  GMRES_PK_MGS = 4,       /* one MGS step h_ij = w . v_i, w -= h_ij v_i */
  GMRES_PK_RESIDUAL = 5,  /* float64 restart residual z = b - A x */
  GMRES_PK_UPDATE = 6,    /* float64 update x += V y (Z y) */
  GMRES_PK_REDUCE = 7,    /* per-system reductions, Givens step, back-solve (latency-bound) */
  GMRES_PK_PRECOND = 8,   /* z_j = M v_j */
  GMRES_PK_ENCODE = 9,    /* 2-byte encoding of a basis vector; orthogonality monitor */
  GMRES_PK_COUNT = 10
};
typedef struct {
  double ms;          /* all launches */
  double ms_active;   /* launches that did work */
  double bytes;       /* algorithmic bytes of the launches that did work */
  int64_t launches;
  int64_t active;
} gmres_kernel_profile;
int gmres_solve_profiled(gmres_handle h, const double* b, double* x, gmres_result* res,
                         gmres_kernel_profile* prof, gmres_kernel_profile* by_col);
/* by_col (HOST, may be NULL): GMRES_PK_COUNT x m entries, entry f * m + j
 * holding family f's launches at Arnoldi column j (the launches of a
 * cycle's start and end, column -1, are in prof only). */

/* The persistent batch schedule's SpMV tuner.  *variant = the SpMV variant
 * the handle's persistent kernel runs (GMRES_PSPMV_*); probe_us (HOST, 3
 * entries, may be NULL) = the tuner's probe time of each variant in
 * microseconds (-1: not probed): one launch of the real kernel over the
 * largest system of each size class for a few Arnoldi steps.  out (HOST, at
 * most cap entries) = the size classes (systems with the same rows per thread
 * of the persistent kernel, n <= 1024 x rows_per_thread): how many systems,
 * the largest n, and the system the probe ran for the class; *count = the
 * number of classes.  ESTATE on a handle that does not run the persistent
 * schedule. */
typedef struct {
  int32_t rows_per_thread;
  int32_t systems;
  int32_t largest_n;
  int32_t probe_system;
} gmres_tune_class;
int gmres_batch_tuning(gmres_handle h, int32_t* variant, double* probe_us, gmres_tune_class* out, int32_t cap,
                       int32_t* count);

/* Launch configuration the solver uses for kernel family `family`
 * (GMRES_PK_SPMV .. GMRES_PK_UPDATE) at Arnoldi column j (0 <= j < m), for
 * the measurement report: *grid workgroups of *block threads; *per_cu = the
 * resident workgroups per compute unit the persistent basis passes size
 * their grid for (grid = per_cu x compute units, capped at the row tiles),
 * 0 for kernels with one workgroup per row block or tile; *basis_align =
 * the largest power of two (up to 2 MiB) dividing the basis allocation's
 * device address.  Any output may be NULL.  ESTATE on the persistent batch
 * schedule. */
int gmres_launch_config(gmres_handle h, int32_t family, int32_t j, int32_t* grid, int32_t* block,
                        int32_t* per_cu, int64_t* basis_align);

/* The Arnoldi SpMV the handle runs, as the autotuner (or the options) left
 * it, for the measurement report: *format = GMRES_SPMV_CSR, GMRES_SPMV_SELL
 * or GMRES_SPMV_SELL16; *block_nnz = the nonzeros per CSR row block (also used by
 * the residual and preconditioner products); *xcd_remap = 1 when consecutive
 * workgroups are mapped onto one XCD; *fin_merged = 1 when the finaliser of
 * Arnoldi step j (column j of H, the Givens step, the decode scale of
 * v_{j+1}) runs in the same launch as the product A v_{j+1}, which then
 * stores w unscaled and leaves the decode scale to the passes that read w
 * first (the first two CGSR projections, in their k_mdot_ds / k_axpy_mdot_ds
 * / k_axpy_mdot64_ds kernels; the first two MGS steps and, at j = 0, the
 * last MGS pass): sliced ELL product, CGSR with m <= 64 or MGS, no
 * preconditioner, a 4- or 8-byte basis (not a float64 product into a
 * float32 w), no orthogonality monitor.  The solve is the same bit for bit
 * either way.  Any output may be NULL.  ESTATE on the persistent batch
 * schedule. */
int gmres_spmv_config(gmres_handle h, int32_t* format, int32_t* block_nnz, int32_t* xcd_remap,
                      int32_t* fin_merged);

#ifdef __cplusplus
}
#endif

#endif /* GMRES_H_ */

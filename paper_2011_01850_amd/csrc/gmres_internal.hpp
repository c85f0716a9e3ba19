// Internal declarations shared by the kernels and the host engine of libgmres.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_plan.hpp"  // kBlock, kTile, row_lanes and the host planning tables

namespace gm {

constexpr int kMaxM = 256;
constexpr int kFinBlock = 1024;  // threads of the per-system finalise kernels
constexpr int kHistCap = 4096;
constexpr int kMaxOcc = 8;       // persistent grids of ncu * k workgroups, k = 1..kMaxOcc
constexpr int kMaxPM = 64;       // persistent batch schedule: restart length limit
constexpr int kMaxPR = 64;       //   and rows per thread (systems up to 1024 * 64 rows)
constexpr int kMaxOrthM = 64;    // loss-of-orthogonality monitor: restart length limit

// Storage of the basis / of w: P64 float64 / float64, P32 float32 / float32,
// PBF16 and PF16 2-byte / float32, PL32 (the limited mode) float32 / float64.
enum Prec { P64 = 0, P32 = 1, PBF16 = 2, PF16 = 3, PL32 = 4 };
// w, its dot products and the Arnoldi product are float64
inline bool wide_w(int prec) { return prec == P64 || prec == PL32; }
enum Status { RUNNING = 0, CONVERGED = 1, MAXITER = 2, STALLED = 3 };

// Per-system scalar state, device resident.  Written only by one lane of a
// finalise kernel (or of a system's first workgroup); every other workgroup
// only reads `active` / `status`.
struct SysState {
  int32_t active;       // the current Arnoldi cycle continues
  int32_t status;       // Status
  int32_t k;            // Arnoldi steps completed in the current cycle
  int32_t need_update;  // the cycle has a correction to apply
  int64_t iters;        // inner iterations, all cycles
  int64_t restarts;     // corrections applied
  double bnorm;         // ||b||_2
  double beta;          // restart residual norm of the current cycle
  double rel;           // beta / bnorm
  double best_beta;
  double prev_beta;
  double wnorm_pre;     // ||A v_j|| before orthogonalisation (breakdown test)
  int32_t no_progress;
  int32_t precond_on;
  int32_t fallback_used;
  int32_t first_stall;  // -1 until seen (first cycle only)
  int32_t kk;           // columns kept by the back-solve
  int32_t nhist;
  int32_t cycle;        // cycles started
  int32_t force;        // timing harness: run gated kernels regardless of state
  float enc_f;          // encode factor of the next 2-byte basis vector
  int32_t klimit;       // two-stage restarts: the first cycle's length (0 until it ends)
  double orth_fro2;     // loss-of-orthogonality monitor: ||S_k||_F^2 of the current cycle
  double orth_norm;     //   and the last norm it compared with the threshold
  double bnorm_p;       // ||M^-1 b||_2 (left preconditioning), else ||b||_2
};

// Work split of a persistent basis pass with G workgroups: workgroup b owns
// the contiguous tile range [b T / G, (b+1) T / G), cut at system
// boundaries into segments; every segment writes one partial row.
struct SegTab {
  int32_t G;               // workgroups
  int32_t nseg;            // segments (= partial rows; column stride of the partial table)
  const int32_t* bseg0;    // [G + 1] first segment of each workgroup
  const int32_t* seg_t0;   // first tile of each segment
  const int32_t* seg_nt;   // tiles of each segment
  const int32_t* seg_sys;  // system of each segment
  const int32_t* sys_sg0;  // first segment of each system
  const int32_t* sys_nsg;  // segments of each system
};

// Everything a kernel needs, passed by value.
struct KArgs {
  int32_t S;        // systems
  int32_t m;        // restart length
  int64_t ld;       // padded rows over all systems: column stride of V, Z, w
  int32_t ntile;    // kTile-row tiles over all systems
  int32_t nrb;      // SpMV row blocks over all systems
  int32_t ps;       // quantities per partial row (m + 3)
  int32_t prec;     // Prec of the Arnoldi process
  int32_t precond;  // 0 none, 1 Jacobi, 2 SPAI
  int32_t ortho;    // 0 MGS, 1 CGSR
  int32_t spmv_budget;  // nnz per SpMV row block (streaming mode)
  int32_t xcd_remap;    // map consecutive blocks onto one XCD
  int32_t ncu;          // compute units of the device
  int32_t vsys;         // basis layout: 0 = column stride ld over all systems,
                        // 1 = one block of (m+1) padded columns per system (persistent batch)
  // matrix: concatenated systems, global row and column numbering
  const int32_t* rp;
  const int32_t* ci;
  const double* a64;    // float64 values (COPY storage), else null
  const float* a32;     // float32 copy (COPY storage, when the Arnoldi product reads float32 values)
  int32_t arn64;        // 1: the Arnoldi product reads the float64 values (else the float32 ones)
  const uint32_t* ahi;  // SPLIT storage: high and low 32-bit words of the float64 values
  const uint32_t* alo;
  int32_t asplit;       // 1: SPLIT storage
  const float* mval;   // SPAI values (float32, A's pattern)
  // The preconditioner computes in float32 (pc64 = 0: the mixed modes, and
  // the float64 solver with a float32 preconditioner) or float64 (pc64 = 1:
  // the float64 solver); its output Z is float64 in the float64 solver
  // (z64 = 1), else float32.
  int32_t pc64;
  int32_t z64;
  int32_t left;        // 1: M^-1 applied on the left (r = M^-1 (b - A x), w = M^-1 A v_j); Z unused
  void* ptmp;          // left preconditioning with the learned M: the product's output (ld rows of w's type)
  const float* dinv;   // Jacobi: 1 / a_ii (float32)
  const double* dinv64;  //   (float64)
  const float* ilu32;  // ILU(0) factors on A's pattern (float32): L below the diagonal, U the rest
  const float* iludinv;  // 1 / u_ii
  const double* ilu64;   // the same factors and 1 / u_ii in float64
  const double* iludinv64;
  const int32_t* diagpos;  // index of each row's diagonal entry (padding rows: their empty start)
  void* ilu_v;         // ILU application: the scaled v_j and three work vectors (ld rows each,
  void* ilu_b[3];      //   float64 when pc64, else float32)
  int32_t ilu_sl, ilu_su;  // sweeps on L and on U
  // sliced ELL copy of the Arnoldi product's values (64-row slices, entry k
  // of a slice's rows contiguous), used instead of the row blocks when every
  // row has fewer than 2 kRowLanePer entries (so its canonical sum is the
  // plain sum in storage order) and the autotuner or the option picks it
  int32_t use_sell;
  int32_t wsc_defer;        // the Arnoldi product stores A v_j unscaled; projections 1 and 2 apply
                            // v_j's decode scale as they load w (the product then runs beside the
                            // finaliser of step j - 1, which computes that scale)
  const void* sell_val;     // float32 or float64 (the values the Arnoldi product reads)
  const int32_t* sell_col;  // 32-bit columns, or
  const int16_t* sell_dcol; //   16-bit offsets from the row (the other is null)
  const int32_t* sell_off;  // first entry of each slice [ld / 64 + 1]
  const uint8_t* sell_len;  // row lengths
  const int32_t* rb;       // row-block first rows [nrb + 1]
  const int32_t* rb_p;     // row pointer at each row-block start [nrb + 1]
  const int32_t* rb_sys;   // system of each row block
  const int32_t* rb_lanes; // lanes per row of each row block: max row_lanes over its rows
  const int32_t* sys_rb0;  // first row block of each system
  const int32_t* sys_nrb;
  const int32_t* tile_sys;  // system of each tile
  const int32_t* sys_t0;    // first tile of each system
  const int32_t* sys_nt;    // tiles of each system
  const int64_t* sys_row0;  // first row of each system
  const int32_t* sys_n;
  SegTab seg[kMaxOcc];      // seg[k - 1]: the split for G = k * ncu workgroups
  // vectors (ld rows each)
  void* V;        // m+1 basis columns, storage per prec
  void* Z;        // m preconditioned columns (flexible form): double when z64, else float
  void* w;        // work vector: double (P64, PL32) or float
  double* x;      // iterate
  double* b;      // right-hand side
  double* zres;   // float64 restart residual (ld rows)
  // scratch: column-major partial tables (quantity q of row k at q * rows + k)
  double* part;
  double* part2;  // second table: MGS alternates between the two
  SysState* st;
  double* H;      // rotated Hessenberg, (m+1) x m per system, column-major
  double* Hbar;   // unrotated copy
  double* cs;     // rotations alpha_i
  double* sn;     // rotations beta_i
  double* s;      // least-squares right-hand side, m+1
  double* y;      // correction coefficients, m
  double* sc;     // decode scale per basis vector, m+1
  double* hacc;   // raw column of H under construction, m+2
  double* h1;     // first CGS projection, m+2
  double* coef;   // coefficients of the running axpy pass, m+2
  double* ares;   // Arnoldi residual per step of the current cycle, m+1
  double* hist;   // restart residual history, kHistCap per system
  // options
  double tol;
  double* ou;      // loss-of-orthogonality monitor, per system (m+1)^2 each: U = strictly upper
  double* os;      //   part of V^T V and S = (I + U)^-1 U, column-major
  double* ocol;    //   the new column of U, (m+1) per system
  double restart_improve;
  double orth_restart;      // loss-of-orthogonality trigger (0 = off)
  int32_t orth_norm;        // 0 spectral, 1 Frobenius
  int32_t restart_repeat;   // two-stage strategy
  int32_t restart_on_stall; // stall-triggered restarts
  int64_t max_iters;
  int32_t stall_cycles;
  int32_t stall_win;  // max(1, ceil(0.05 m))
  // persistent batch schedule: the ELL copy of the float32 values that the
  // ELL variant of its Arnoldi SpMV reads
  const float* ell_val;     // system s: ell_w[s] slices of sys_nt[s] * kTile rows from ell_off[s]
  const uint16_t* ell_col;  //   column minus the system's first row
  const uint8_t* ell_len;   // row lengths (global rows)
  const int64_t* ell_off;
  const int32_t* ell_w;     // 0: the system has no ELL copy
};

// Arnoldi SpMV of the persistent batch kernel (one thread per row, R rows
// per thread), one kernel per variant, chosen per batch by the create-time
// tuner.  Every variant sums a row's products in storage order, so the
// choice changes speed only, never a result bit.
//   PV_CSR8  CSR, a row's entries loaded in groups of 8
//   PV_CSR4  CSR, groups of 4
//   PV_ELL16 ELL: entry k of every row of the system in one slice (loads
//            coalesced across the workgroup), 16-bit columns local to the
//            system, one byte of row length (systems up to 65,536 rows and
//            rows up to 255 entries)
enum PersistentSpmv { PV_CSR8 = 0, PV_CSR4 = 1, PV_ELL16 = 2, PV_COUNT = 3 };

// ---------------------------------------------------------------- launchers
// Each launcher enqueues its kernels on `st` and returns hipGetLastError().
// The basis passes are followed by the kernel that completes them unless
// with_fin is false (kernel timing).
hipError_t launch_spmv_arnoldi(const KArgs& a, int j, hipStream_t st);   // w = A v_j or A z_j
hipError_t launch_precond(const KArgs& a, int j, hipStream_t st);        // z_j = M v_j
hipError_t launch_residual(const KArgs& a, hipStream_t st, bool with_fin = true);  // z = b - A x
hipError_t launch_encode(const KArgs& a, int col, hipStream_t st);       // store w as basis column
hipError_t launch_cgs_pass1(const KArgs& a, int j, hipStream_t st, bool with_fin = true);
hipError_t launch_cgs_pass2(const KArgs& a, int j, hipStream_t st, bool with_fin = true);
hipError_t launch_final_pass(const KArgs& a, int j, hipStream_t st, bool with_fin = true);
// the finaliser of step j_fin and the Arnoldi product of column j_fin + 1 in
// one launch (sliced ELL product, wsc_defer set)
hipError_t launch_spmv_fin(const KArgs& a, int j_fin, hipStream_t st);
hipError_t launch_mgs_dot(const KArgs& a, int j, int i, hipStream_t st);
// Loss-of-orthogonality monitor after step j: column j+1 of U and S, the
// norm of S, and the end of the cycle when it reaches the threshold.
hipError_t launch_orth_check(const KArgs& a, int j, hipStream_t st);
hipError_t launch_backsolve(const KArgs& a, hipStream_t st);
// the kernel that completes CGS projection 2 at column j (timing)
hipError_t launch_finalize_pass2(const KArgs& a, int j, hipStream_t st);
// Left preconditioning: w <- M^-1 w on the systems whose cycle runs with the
// preconditioner on (every system while the state's force flag is set);
// launch_left_start: after the restart residual, M^-1 z, its norm and the
// cycle's s_1 and first decode scale; launch_left_bnorm: ||M^-1 b|| at the
// start of a solve (w is overwritten).
hipError_t launch_left_apply(const KArgs& a, hipStream_t st);
hipError_t launch_left_start(const KArgs& a, hipStream_t st);
hipError_t launch_left_bnorm(const KArgs& a, hipStream_t st);
// The completing reductions on their own (the in-solve profile launches each
// pass without its reduction, then these): the residual's norm and stop
// test, projection 1's coefficients, and the end-of-step finaliser.
// Launch configuration of a kernel family (GMRES_PK_* numbering, 0-6) at
// column j: workgroups, threads per workgroup, and for the persistent
// passes the resident workgroups per CU their grid is sized for (else 0).
hipError_t launch_config(const KArgs& a, int family, int j, int32_t* grid, int32_t* block, int32_t* per_cu);
hipError_t launch_residual_finish(const KArgs& a, hipStream_t st);
hipError_t launch_finalize_pass1(const KArgs& a, int j, hipStream_t st);
hipError_t launch_finalize_final(const KArgs& a, int j, hipStream_t st);
hipError_t launch_update(const KArgs& a, hipStream_t st);
hipError_t launch_bnorm(const KArgs& a, hipStream_t st);
hipError_t launch_init_state(const KArgs& a, hipStream_t st);
hipError_t launch_set_force(const KArgs& a, int on, hipStream_t st);
hipError_t launch_check_cols(const KArgs& a, int32_t* bad, hipStream_t st);
hipError_t launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t st);
// float64 values -> high and low 32-bit words (SPLIT storage), and back
hipError_t launch_split_words(const double* src, uint32_t* hi, uint32_t* lo, int64_t n, hipStream_t st);
hipError_t launch_merge_words(const uint32_t* hi, const uint32_t* lo, double* dst, int64_t n, hipStream_t st);
// sum of squares of v[0, n) as nblk partials (part[0, nblk)); out = float32(r * f)
constexpr int kSumsqBlocks = 1024;
hipError_t launch_sumsq(const double* v, int64_t n, double* part, int nblk, hipStream_t st);
hipError_t launch_scale_f32(const double* r, int64_t n, double f, float* out, hipStream_t st);
hipError_t launch_jacobi_setup(const KArgs& a, float* dinv, double* dinv64, hipStream_t st);
// ILU(0) factorisation of the rows rows[0, count) (one dependency level), in place on lu
hipError_t launch_ilu_factor(const KArgs& a, double* lu, const int32_t* rows, int32_t count, hipStream_t st);
// z = U^-1 L^-1 ilu_v by the configured sweeps, the result in dst
hipError_t launch_ilu_apply(const KArgs& a, void* dst, hipStream_t st);
// float32 factors and 1/u_ii from the float64 factors
hipError_t launch_ilu_finish(const KArgs& a, const double* lu, float* lu32, float* dinv, double* dinv64,
                             hipStream_t st);
hipError_t launch_spmv_plain(const KArgs& a, int prec, const void* x, void* y, hipStream_t st);
// The sliced ELL copy of A (values from `vals`, float32 when v32 else float64)
hipError_t launch_build_sell(const KArgs& a, const void* vals, int v32, void* sv, int32_t* sc, int16_t* sd,
                             uint8_t* sl, hipStream_t st);
hipError_t launch_residual_plain(const KArgs& a, const double* b, const double* x, double* r,
                                 hipStream_t st);
hipError_t launch_encode_plain(int prec, int64_t n, const float* w, float f, void* out,
                               hipStream_t st);
hipError_t launch_absmax(const float* w, int64_t n, float* part, int nblk, hipStream_t st);
hipError_t launch_decode_column(const KArgs& a, int sys, int col, double* out, hipStream_t st);
hipError_t launch_shift_cols(const int32_t* src, int32_t* dst, int64_t nnz, int32_t shift,
                             hipStream_t st);
hipError_t launch_gather(const double* const* src, double* dst, const int64_t* row0,
                         const int32_t* n, int S, int64_t maxn, hipStream_t st);
hipError_t launch_scatter(const double* src, double* const* dst, const int64_t* row0,
                          const int32_t* n, int S, int64_t maxn, hipStream_t st);
// One workgroup per system, systems taken from `order` through `counter`
// (cleared by this call), float32 MGS Arnoldi; basis in layout vsys = 1.
// One workgroup per system, systems taken from `order` (a.S entries) through
// `counter` (cleared by this call), float32 MGS Arnoldi; basis in layout
// vsys = 1; pv: the Arnoldi SpMV variant (PersistentSpmv).
hipError_t launch_batch_persistent(const KArgs& a, const int32_t* order, int32_t* counter, int pv, hipStream_t st);
// The ELL copy of system s (one thread per row): values from a.a32, local
// columns, lengths; w = ELL width of s (its longest row).
hipError_t launch_build_ell(const KArgs& a, int s, int64_t row0, int n, int w, int64_t off, int pn,
                            float* val, uint16_t* col, uint8_t* len, hipStream_t st);
// Queries, once per process, how many workgroups of each persistent basis
// pass of `prec` fit on one CU.  Must run before any graph capture.
hipError_t prepare_occupancy(int prec);

// Device blocks of the handles (device_cache.cpp): cache_alloc takes a
// block of at least `bytes` on the current device (a released block of the
// same rounded size, else a new one; nullptr when out of memory) and stores
// the rounded size in *rounded; cache_free returns it for reuse (all work
// that reads it must be complete); cache_release_all frees every released
// block and returns how many bytes that was.
void* cache_alloc(size_t bytes, size_t* rounded);
void cache_free(void* p);
size_t cache_release_all();

}  // namespace gm

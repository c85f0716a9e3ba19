// Internal declarations shared by the kernels and the host engine of libgmres.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gm {

// Rows per reduction chunk: one workgroup of kBlock threads owns kChunk
// consecutive rows of one system for every basis pass.  Systems are padded
// to a multiple of kChunk rows (padding rows of the basis and of w are zero
// and stay zero), so the passes need no tail handling.
constexpr int kBlock = 256;
constexpr int kChunk = 2048;
constexpr int kRowsPerThread = kChunk / kBlock;  // 8
constexpr int kMaxM = 256;
constexpr int kFinBlock = 1024;  // threads of the per-system finalise kernels
constexpr int kHistCap = 4096;

enum Prec { P64 = 0, P32 = 1, PBF16 = 2, PF16 = 3 };
enum Status { RUNNING = 0, CONVERGED = 1, MAXITER = 2, STALLED = 3 };

// Per-system scalar state, device resident.  Written only by single-lane
// finalisers (the last workgroup of a pass) and by the small per-system
// kernels; every other workgroup only reads `active` / `status`.
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
  float pad_;
};

// Everything a kernel needs, passed by value.
struct KArgs {
  int32_t S;        // systems
  int32_t m;        // restart length
  int64_t ld;       // padded rows over all systems: column stride of V, Z, w
  int32_t nchunk;   // kChunk-row chunks over all systems
  int32_t nrb;      // SpMV row blocks over all systems
  int32_t ps;       // row stride of the partials table
  int32_t prec;     // Prec of the Arnoldi process
  int32_t precond;  // 0 none, 1 Jacobi, 2 SPAI
  int32_t ortho;    // 0 MGS, 1 CGSR
  int32_t spmv_budget;  // nnz per SpMV row block (streaming mode)
  int32_t xcd_remap;    // map consecutive blocks onto one XCD
  // matrix: concatenated systems, global row and column numbering
  const int32_t* rp;
  const int32_t* ci;
  const double* a64;
  const float* a32;
  const float* mval;   // SPAI values (float32, A's pattern)
  const float* dinv;   // Jacobi: 1 / a_ii
  const int32_t* rb;       // row-block first rows [nrb + 1]
  const int32_t* rb_sys;   // system of each row block
  const int32_t* ch_sys;   // system of each chunk
  const int32_t* sys_rb0;  // first row block of each system
  const int32_t* sys_nrb;
  const int32_t* sys_ch0;  // first chunk of each system
  const int32_t* sys_nch;
  const int64_t* sys_row0;  // first row of each system
  const int32_t* sys_n;
  // vectors (ld rows each)
  void* V;        // m+1 basis columns, storage per prec
  float* Z;       // m preconditioned columns (flexible form)
  void* w;        // work vector: double (P64) or float
  double* x;      // iterate
  double* b;      // right-hand side
  // two-level reduction: each workgroup writes one row of `part`; the last
  // workgroup of a group reduces the group's rows into one row of `part2`;
  // the last group of a system reduces those rows and finalises the system
  const int32_t* ch_grp;    // group of each chunk
  const int32_t* ch_gfirst; // first chunk of each chunk group
  const int32_t* ch_gn;     // chunks in each chunk group
  const int32_t* sys_cg0;   // first chunk group of each system
  const int32_t* sys_cng;   // chunk groups of each system
  const int32_t* rb_grp;    // same for the SpMV row blocks
  const int32_t* rb_gfirst;
  const int32_t* rb_gn;
  const int32_t* sys_rg0;
  const int32_t* sys_rng;
  // scratch
  double* part;    // level-1 partials [max(nchunk, nrb)][ps]
  double* part2;   // level-2 partials [max(groups)][ps]
  uint32_t* gcnt;  // group counters
  uint32_t* cnt;   // system counters
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
  double restart_improve;
  int64_t max_iters;
  int32_t stall_cycles;
  int32_t stall_win;  // max(1, ceil(0.05 m))
};

// ---------------------------------------------------------------- launchers
// Each launcher enqueues one kernel on `st` and returns hipGetLastError().
hipError_t launch_spmv_arnoldi(const KArgs& a, int j, hipStream_t st);   // w = A v_j or A z_j
hipError_t launch_precond(const KArgs& a, int j, hipStream_t st);        // z_j = M v_j
hipError_t launch_residual(const KArgs& a, hipStream_t st, bool with_fin = true);             // z = b - A x, start cycle
hipError_t launch_encode(const KArgs& a, int col, hipStream_t st);       // 2-byte store of w
hipError_t launch_cgs_pass1(const KArgs& a, int j, hipStream_t st, bool with_fin = true);
hipError_t launch_cgs_pass2(const KArgs& a, int j, hipStream_t st, bool with_fin = true);
hipError_t launch_final_pass(const KArgs& a, int j, int i0, hipStream_t st, bool with_fin = true);
hipError_t launch_mgs_dot(const KArgs& a, int j, int i, hipStream_t st, bool with_fin = true);
hipError_t launch_backsolve(const KArgs& a, hipStream_t st);
// mode: 0 CGS projection 1, 1 projection 2, 2 Givens step, 3 MGS dot, 4 residual
hipError_t launch_finalize(const KArgs& a, int mode, int j, int i, hipStream_t st);
hipError_t launch_update(const KArgs& a, hipStream_t st);
hipError_t launch_bnorm(const KArgs& a, hipStream_t st);
hipError_t launch_init_state(const KArgs& a, hipStream_t st);
hipError_t launch_set_force(const KArgs& a, int on, hipStream_t st);
hipError_t launch_check_cols(const KArgs& a, int32_t* bad, hipStream_t st);
hipError_t launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t st);
hipError_t launch_jacobi_setup(const KArgs& a, float* dinv, hipStream_t st);
hipError_t launch_spmv_plain(const KArgs& a, int prec, const void* x, void* y, hipStream_t st);
hipError_t launch_residual_plain(const KArgs& a, const double* b, const double* x, double* r,
                                 hipStream_t st);
hipError_t launch_sumsq(const double* v, int64_t n, double* part, int nblk, hipStream_t st);
hipError_t launch_encode_plain(int prec, int64_t n, const float* w, float f, void* out,
                               hipStream_t st);
hipError_t launch_absmax(const float* w, int64_t n, float* part, int nblk, hipStream_t st);
hipError_t launch_decode_column(const KArgs& a, int sys, int col, double* out, hipStream_t st);
hipError_t launch_shift_cols(const int32_t* src, int32_t* dst, int64_t nnz, int32_t shift,
                             hipStream_t st);
hipError_t launch_shift_rowptr(const int32_t* src, int32_t* dst, int64_t n, int32_t shift,
                               hipStream_t st);
hipError_t launch_gather(const double* const* src, double* dst, const int64_t* row0,
                         const int32_t* n, int S, int64_t maxn, hipStream_t st);
hipError_t launch_scatter(const double* src, double* const* dst, const int64_t* row0,
                          const int32_t* n, int S, int64_t maxn, hipStream_t st);

}  // namespace gm

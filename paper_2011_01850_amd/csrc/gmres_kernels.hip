// HIP kernels of restarted GMRES(m) for gfx950 (wave64).
//
// Method: Algorithm 1 of Lindquist, Luszczek, Dongarra (arXiv 2011.01850):
// float64 residual and update, float32 (or 2-byte-stored) Arnoldi process,
// MGS or CGSR (two classical projections) orthogonalisation, Givens QR of
// the Hessenberg matrix in float64.
//
// Execution model.  Every system of a handle is a contiguous, zero-padded
// range of 256-row tiles.  A basis pass is a persistent grid sized to the
// kernel's occupancy: each workgroup streams a contiguous, balanced range of
// tiles (one row per thread) and writes one partial row per system segment
// it touches; the next kernel (a small per-system finalise, or the next MGS
// step itself) reduces those partials in a fixed order.  Matrix passes run
// one workgroup per CSR row block.  All reductions are deterministic: per-lane
// sums, a fixed in-wave butterfly, a fixed cross-wave order and fixed-order
// sums of the partials; no floating-point atomics.  Kernels of a cycle are
// gated by the device-side `active` flag of their system, so a whole restart
// cycle can be enqueued (or captured in one graph) without host round trips.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "gmres_internal.hpp"

namespace gm {

struct bf16_t {
  uint16_t b;
};
using f16_t = _Float16;

template <typename T>
struct AccOf {
  using type = float;
};
template <>
struct AccOf<double> {
  using type = double;
};

// A's values in SPLIT storage: HiW reads the high 32-bit word of each
// float64 value (the value truncated to 20 significand bits) as float32;
// HiLoW reads the high word and the low word at the same index of the
// separate low-word array, i.e. the float64 value itself.
struct HiW {
  uint32_t w;
};
struct HiLoW {
  uint32_t w;
};
template <>
struct AccOf<HiLoW> {
  using type = double;
};
// Accumulation type of a kernel that reads TIn and writes TOut: float64
// whenever the written vector is float64 (the limited precision mode keeps
// w, its dot products and the Arnoldi product's sums in float64 over a
// float32 basis and a float32 copy of A), else that of what it reads.
template <typename TIn, typename TOut>
using AccFor = typename std::conditional<sizeof(TOut) == 8, double, typename AccOf<TIn>::type>::type;
__device__ __forceinline__ float hi_value(uint32_t h) { return (float)__hiloint2double((int)h, 0); }
__device__ __forceinline__ double hilo_value(uint32_t h, uint32_t l) { return __hiloint2double((int)h, (int)l); }

// Value k of A for the SpMV (element type TA, see above).
template <typename TA>
__device__ __forceinline__ typename AccOf<TA>::type a_value(const KArgs& a, const TA* vals, int k) {
  if constexpr (std::is_same<TA, HiW>::value)
    return hi_value(vals[k].w);
  else if constexpr (std::is_same<TA, HiLoW>::value)
    return hilo_value(vals[k].w, a.alo[k]);
  else
    return (typename AccOf<TA>::type)vals[k];
}

__device__ __forceinline__ float ldv(float v) { return v; }
__device__ __forceinline__ double ldv(double v) { return v; }
__device__ __forceinline__ float ldv(bf16_t v) { return __uint_as_float(((uint32_t)v.b) << 16); }
__device__ __forceinline__ float ldv(f16_t v) { return (float)v; }

template <typename T>
__device__ __forceinline__ T stv(float v);
template <>
__device__ __forceinline__ float stv<float>(float v) { return v; }
template <>
__device__ __forceinline__ bf16_t stv<bf16_t>(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t{(uint16_t)((u >> 16) | 0x40u)};  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return bf16_t{(uint16_t)(u >> 16)};
}
template <>
__device__ __forceinline__ f16_t stv<f16_t>(float v) { return (f16_t)v; }  // v_cvt_f16_f32: RNE

// The stored 2-byte value is round(float32(w * f)): the product is its own
// float32 rounding, never fused with the conversion (v_fma_mix would round
// the exact product once).
__device__ __forceinline__ float mul_rn(float a, float b) {
  float t = a * b;
  asm volatile("" : "+v"(t));
  return t;
}
// A product that is never fused into a following add (its multiply carries
// no contraction flag; no scheduling fence either).
__device__ __forceinline__ float mul_nofuse(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ double mul_nofuse(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

template <typename T>
__device__ __forceinline__ T stw(double v);
template <>
__device__ __forceinline__ double stw<double>(double v) { return v; }
template <>
__device__ __forceinline__ float stw<float>(double v) { return (float)v; }

// ------------------------------------------------------------ block helpers

// Stores of the streamed vectors (w, the new basis column, the product's
// output) carry the non-temporal hint: the next kernel reads them from the
// memory-side cache either way, and lines not left dirty in L2 make each
// kernel's end (which writes L2 back) shorter.  2-byte types store plainly.
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  if constexpr (sizeof(T) == 2)
    *p = v;
  else
    __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ int remap_block(int b, int G, int on) {
  // consecutive logical blocks on one XCD: dispatch is round-robin over 8 XCDs
  if (!on) return b;
  const int per = G >> 3, rem = G & 7, x = b & 7, q = b >> 3;
  return x * per + (x < rem ? x : rem) + q;
}


template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Sum over the 256 threads, identical result in every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T red[kBlock / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = red[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}
template <typename T>
__device__ __forceinline__ T block_max(T v) {
  __shared__ T red[kBlock / 64];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = red[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) t = fmax(t, red[i]);
  __syncthreads();
  return t;
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// In-wave reduce-scatter of L column values (L a power of two <= 64):
// afterwards lane l holds the wave-wide sum of column (l >> (6 - log2 L)).
template <int L, typename T>
__device__ __forceinline__ T reduce_scatter(T (&p)[L], int lane) {
  constexpr int P = ilog2c(L);
#pragma unroll
  for (int st = 0; st < P; ++st) {
    const int o = 32 >> st;
    const int half = (L >> st) >> 1;
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int q = 0; q < half; ++q) {
      // select values, not array slots: a conditional lvalue would make the
      // array addressable and push it to scratch memory
      const T lo = p[q], hi = p[q + half];
      const T keep = up ? hi : lo;
      const T send = up ? lo : hi;
      p[q] = keep + __shfl_xor(send, o);
    }
  }
  T v = p[0];
#pragma unroll
  for (int o = 32 >> P; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum (or maximum) of p[0, n) in a fixed order; called by every thread of
// the block (up to kFinBlock threads), the result is returned in all of them.
// Partial tables are column-major (one contiguous column per quantity), so
// the loads here are contiguous.
template <bool kMax>
__device__ double reduce_col(const double* p, int n) {
  __shared__ double sh[kFinBlock / 64];
  const int t = threadIdx.x, NT = blockDim.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int r = t;
  for (; r + 3 * NT < n; r += 4 * NT) {
    if (kMax) {
      a0 = fmax(a0, p[r]); a1 = fmax(a1, p[r + NT]); a2 = fmax(a2, p[r + 2 * NT]); a3 = fmax(a3, p[r + 3 * NT]);
    } else {
      a0 += p[r]; a1 += p[r + NT]; a2 += p[r + 2 * NT]; a3 += p[r + 3 * NT];
    }
  }
  for (; r < n; r += NT) a0 = kMax ? fmax(a0, p[r]) : a0 + p[r];
  double v = kMax ? fmax(fmax(a0, a1), fmax(a2, a3)) : (a0 + a1) + (a2 + a3);
  v = kMax ? wave_max(v) : wave_sum(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double tot = sh[0];
  for (int w = 1; w < NT / 64; ++w) tot = kMax ? fmax(tot, sh[w]) : tot + sh[w];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ bool gated(const KArgs& a, int s) {
  const SysState& S = a.st[s];
  return S.active != 0 || S.force != 0;
}

// The gate of system 0, read at a kernel's start from an address that needs
// no other load (the single-system case).
__device__ __forceinline__ int gate0(const KArgs& a) { return a.st[0].active | a.st[0].force; }

// The gate test of a kernel whose first loads do not depend on it: `on0` is
// gate0(), and `issued` (any non-negative value loaded beside it) ties those
// loads to the test, so they are in flight together rather than each
// waiting for the gate.
__device__ __forceinline__ bool gated_now(const KArgs& a, int s, int on0, int issued) {
  const bool on = a.S == 1 ? on0 != 0 : gated(a, s);
  return on & (issued >= 0);
}

__device__ __forceinline__ double unit_roundoff(int prec) {
  return prec == P64 ? 0x1p-53 : 0x1p-24;
}

// e with vmax * 2^e in (T/2, T]; T = 2^15 for half, 1 for bfloat16.
__device__ __forceinline__ int scale_exp(double vmax, int prec) {
  if (!(vmax > 0.0) || !isfinite(vmax)) return 0;
  int p;
  const double f = frexp(vmax, &p);
  return (prec == PF16 ? 15 : 0) - p + (f == 0.5 ? 1 : 0);
}

__device__ __forceinline__ void givens(double a, double b, double& c, double& s) {
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double rho = hypot(a, b);
  c = a / rho;
  s = b / rho;
}

// ------------------------------------------------------------- finalisers
// All run in the last block of a pass; `red` holds the reduced partials.

// Givens update of column j, restart / stop decisions (one lane).
// Called by every thread of the finalising workgroup: the column and the
// earlier rotations are staged in LDS in parallel, one lane runs the
// sequential rotation chain in registers, and the column is written back in
// parallel.
// Staged inputs of the per-step finaliser (LDS): the unrotated column of H,
// the earlier rotations, and the two history values the tests need.
struct FinShared {
  double hcol[kMaxM + 2], rc[kMaxM], rsn[kMaxM];
  double svj, arJ;
  int ok;
};

// Givens update of column j, restart / stop decisions (one lane), on S, a
// copy of the system's state in LDS that the caller writes back.  The column
// and the rotations are staged (fin_stage) before the partial sums are
// reduced, so their loads overlap; one lane runs the sequential rotation
// chain in registers; the column is written back in parallel.
__device__ void fin_stage(const KArgs& a, int s, int j, FinShared& sh) {
  const int t = threadIdx.x, NT = blockDim.x;
  const int m = a.m, M1 = m + 1, M2 = m + 2;
  const double* hc = a.hacc + (int64_t)s * M2;
  const double* cs = a.cs + (int64_t)s * m;
  const double* sn = a.sn + (int64_t)s * m;
  for (int i = t; i <= j; i += NT) sh.hcol[i] = hc[i];
  for (int i = t; i < j; i += NT) {
    sh.rc[i] = cs[i];
    sh.rsn[i] = sn[i];
  }
  if (t == 0) sh.svj = a.s[(int64_t)s * M1 + j];
  if (t == 1) {
    const int J = j + 1 - a.stall_win;
    sh.arJ = J >= 0 ? a.ares[(int64_t)s * M1 + J] : 0.0;
  }
}

__device__ void fin_step(const KArgs& a, int s, int j, double sumsq, double wmax, SysState& S, FinShared& sh) {
  const int t = threadIdx.x, NT = blockDim.x;
  const int m = a.m, M1 = m + 1;
  double* col = a.H + (int64_t)s * M1 * m + (int64_t)j * M1;
  double* bcol = a.Hbar + (int64_t)s * M1 * m + (int64_t)j * M1;
  double* cs = a.cs + (int64_t)s * m;
  double* sn = a.sn + (int64_t)s * m;
  const double hn = sqrt(sumsq);
  if (t == 0) sh.ok = isfinite(hn) ? 1 : 0;
  __syncthreads();
  for (int i = t; i <= j; i += NT)
    if (!isfinite(sh.hcol[i])) sh.ok = 0;
  __syncthreads();
  const bool finite = sh.ok != 0;
  if (t == 0) {
    if (!finite) {
      // drop the column; the cycle ends with the finite part of the basis
      if (a.restart_repeat && S.klimit == 0 && j > 0) S.klimit = j;
      S.k = j;
      S.need_update = j > 0 ? 1 : 0;
      S.active = 0;
      if (a.precond != 0 && S.precond_on) {
        S.precond_on = 0;
        S.fallback_used = 1;
      }
    } else {
      double* sv = a.s + (int64_t)s * M1;
      double* sc = a.sc + (int64_t)s * M1;
      double* ar = a.ares + (int64_t)s * M1;
      // apply the previous rotations; only the running entry is carried
      double cur = sh.hcol[0];
      for (int i = 0; i < j; ++i) {
        const double nxt = sh.hcol[i + 1];
        sh.hcol[i] = sh.rc[i] * cur + sh.rsn[i] * nxt;
        cur = -sh.rsn[i] * cur + sh.rc[i] * nxt;
      }
      double c, sg;
      givens(cur, hn, c, sg);
      cs[j] = c;
      sn[j] = sg;
      const double sj = sh.svj;
      sv[j + 1] = -sg * sj;
      sv[j] = c * sj;
      sh.hcol[j] = c * cur + sg * hn;
      sh.hcol[j + 1] = 0.0;
      S.iters += 1;
      S.k = j + 1;
      S.need_update = 1;
      const double res = fabs(sg * sj);
      ar[j + 1] = res;
      const int J = j + 1 - a.stall_win;  // the stall window's start (sh.arJ = |s_{J+1}|)
      if (S.cycle == 1 && S.first_stall < 0) {
        if (J >= 0 && res > sh.arJ / 1.001) S.first_stall = J;
      }
      const double bd = 16.0 * (double)(j + 1) * unit_roundoff(a.prec);
      // restart triggers: the improvement threshold (first cycle only under
      // the two-stage strategy), the first cycle's length (two-stage), a
      // stalled Arnoldi residual
      const bool first_stage = !a.restart_repeat || S.klimit == 0;
      // (left preconditioning: |s_{j+1}| estimates ||M^-1 (b - A x)||)
      const double est_ref = a.left && S.precond_on ? S.bnorm_p : S.bnorm;
      const bool end = (j + 1 >= m) || !(hn > bd * S.wnorm_pre) || res <= a.tol * est_ref ||
                       S.iters >= a.max_iters ||
                       (a.restart_improve > 0.0 && first_stage && res <= a.restart_improve * S.beta) ||
                       (!first_stage && j + 1 >= S.klimit) ||
                       (a.restart_on_stall && J >= 0 && res > sh.arJ / 1.001);
      if (end && a.restart_repeat && S.klimit == 0) S.klimit = j + 1;
      if (a.prec == PBF16 || a.prec == PF16) {
        if (!end) {
          const int e = scale_exp(wmax / hn, a.prec);
          sc[j + 1] = ldexp(1.0, -e);
          S.enc_f = (float)(ldexp(1.0, e) / hn);
        }
      } else if (hn > 0.0) {
        // w'' is already stored as column j+1; its scale also completes the
        // last cycle's basis when the cycle ends here
        sc[j + 1] = 1.0 / hn;
      }
      S.active = end ? 0 : 1;
    }
  }
  __syncthreads();
  if (finite) {
    const double* hc = a.hacc + (int64_t)s * (m + 2);
    for (int i = t; i <= j; i += NT) bcol[i] = hc[i];
    if (t == 0) bcol[j + 1] = hn;
    for (int i = t; i <= j + 1; i += NT) col[i] = sh.hcol[i];
  }
}

__device__ void fin_residual(const KArgs& a, int s, double sumsq, double zmax) {
  SysState& S = a.st[s];
  const int M1 = a.m + 1;
  S.need_update = 0;
  S.active = 0;
  const double beta = sqrt(sumsq);
  S.beta = beta;
  S.rel = beta / S.bnorm;
  if (S.nhist < kHistCap) a.hist[(int64_t)s * kHistCap + S.nhist] = S.rel;
  S.nhist += 1;
  if (S.force) return;
  if (S.rel <= a.tol) {
    S.status = CONVERGED;
    return;
  }
  if (!isfinite(beta)) {
    S.status = STALLED;
    return;
  }
  if (S.iters >= a.max_iters) {
    S.status = MAXITER;
    return;
  }
  if (beta >= S.best_beta)
    S.no_progress += 1;
  else
    S.no_progress = 0;
  S.best_beta = fmin(S.best_beta, beta);
  if (S.no_progress >= a.stall_cycles) {
    S.status = STALLED;
    return;
  }
  if (a.precond != 0 && S.precond_on && beta > S.prev_beta / 1.001) {
    S.precond_on = 0;
    S.fallback_used = 1;
  }
  S.prev_beta = beta;
  S.k = 0;
  S.cycle += 1;
  a.s[(int64_t)s * M1] = beta;
  a.ares[(int64_t)s * M1] = beta;
  if (a.prec == PBF16 || a.prec == PF16) {
    const int e = scale_exp(zmax / beta, a.prec);
    a.sc[(int64_t)s * M1] = ldexp(1.0, -e);
    S.enc_f = (float)(ldexp(1.0, e) / beta);
  } else {
    a.sc[(int64_t)s * M1] = 1.0 / beta;
  }
  S.active = 1;
}

// ------------------------------------------------------------------ SpMV

enum SpmvMode { SM_ARNOLDI = 0, SM_PRECOND = 1, SM_AZ = 2, SM_RESID = 3, SM_PLAIN = 4, SM_RESID_PLAIN = 5,
                SM_LEFT = 6 };

// Adaptive CSR: a row block is either up to 256 rows whose non-zeros fit
// the streaming budget (products staged in LDS, each row reduced by a
// power-of-two group of lanes) or one long row staged by the whole block.
//
// Every row is summed in the canonical order of row_lanes (lane l of T adds
// the products l, l + T, ... in turn, then a fixed butterfly), so the
// row-block layout (which the autotuner picks) never changes a result.

// 16-byte loads of the matrix arrays.  (The non-temporal hint on these
// streams was measured on the stencil and power-law matrices and never
// gained: the gathers, not the streams, are what the L2 misses.)
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
template <typename V>
__device__ __forceinline__ V ld16(const void* p) {
  return *reinterpret_cast<const V*>(p);
}

template <typename TA, typename TX, typename TY, int MODE>
__global__ __launch_bounds__(kBlock) void k_spmv(KArgs a, const TA* __restrict__ vals,
                                                 const TX* __restrict__ x, TY* __restrict__ y,
                                                 const double* __restrict__ bvec, int j) {
  using ACC = AccFor<TA, TY>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  ACC* prod = reinterpret_cast<ACC*>(smem_raw);
  const int blk = remap_block(blockIdx.x, gridDim.x, a.xcd_remap);
  const int t = threadIdx.x;
  // the block's rows and non-zero range come from tables of their own, so
  // they load together with the system's gate rather than after it
  const int on0 = gate0(a);
  const int s = a.S == 1 ? 0 : a.rb_sys[blk];
  const int r0 = a.rb[blk], r1 = a.rb[blk + 1];
  const int p0 = a.rb_p[blk], p1 = a.rb_p[blk + 1];
  if (MODE == SM_ARNOLDI || MODE == SM_PRECOND || MODE == SM_AZ) {
    if (!gated_now(a, s, on0, p0 | r0)) return;
  } else if (MODE == SM_LEFT) {  // the learned M applied to w (left preconditioning), unscaled
    if (!gated(a, s) || (!a.st[s].precond_on && !a.st[s].force)) return;
  } else if (MODE == SM_RESID) {
    const SysState& S = a.st[s];
    if (S.status != RUNNING && !S.force) return;
  }
  ACC scale = (ACC)1;
  if (MODE == SM_ARNOLDI || MODE == SM_PRECOND) scale = (ACC)a.sc[(int64_t)s * (a.m + 1) + j];
  if (MODE == SM_PRECOND && !a.st[s].precond_on) {
    // preconditioner switched off: z_j = v_j
    for (int r = r0 + t; r < r1; r += kBlock) y[r] = (TY)(scale * (ACC)ldv(x[r]));
    return;
  }
  double zsq = 0.0, zmax = 0.0;
  auto emit = [&](int r, ACC acc) {
    if (MODE == SM_RESID || MODE == SM_RESID_PLAIN) {
      const double z = bvec[r] - (double)acc;
      zsq += z * z;
      zmax = fmax(zmax, fabs(z));
      y[r] = (TY)z;
      if (MODE == SM_RESID) a.zres[r] = z;
    } else {
      st_nt(&y[r], (TY)(acc * scale));
    }
  };
  if (p1 - p0 > a.spmv_budget) {  // one long row: staged chunk by chunk, lanes 0..T-1 of wave 0 add
    const int T = row_lanes(p1 - p0);
    ACC acc = (ACC)0;
    for (int c0 = p0; c0 < p1; c0 += a.spmv_budget) {  // chunks are multiples of T long
      const int c1 = min(p1, c0 + a.spmv_budget);
      for (int k = c0 + t; k < c1; k += kBlock) prod[k - c0] = a_value(a, vals, k) * (ACC)ldv(x[a.ci[k]]);
      __syncthreads();
      if (t < T)
        for (int k = c0 + t; k < c1; k += T) acc += prod[k - c0];
      __syncthreads();
    }
    if (t < 64) {
      for (int o = T >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (t == 0) emit(r0, acc);
    }
  } else {
    // products staged in LDS; indices and values are read as aligned groups
    // of four (16-byte index loads; the matrix arrays carry a zero pad of
    // four entries so a group never leaves them), two groups a thread in
    // flight at once
    const int tpr = a.rb_lanes[blk];
    const int g = t / tpr, l = t % tpr, ng = kBlock / tpr;
    // the first row of this lane group: its range loads beside the matrix
    int rb_ = 0, re_ = 0;
    if (r0 + g < r1) {
      rb_ = a.rp[r0 + g];
      re_ = a.rp[r0 + g + 1];
    }
    const int q0 = p0 & ~3;
    constexpr int kU = 2;
    for (int base = q0 + 4 * t; base < p1; base += 4 * kBlock * kU) {
      i32x4_t c4[kU];
      ACC v4[kU][4];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int k4 = base + u * 4 * kBlock;
        if (k4 >= p1) {
          c4[u] = i32x4_t{0, 0, 0, 0};
          v4[u][0] = v4[u][1] = v4[u][2] = v4[u][3] = (ACC)0;
          continue;
        }
        c4[u] = ld16<i32x4_t>(a.ci + k4);
        if constexpr (std::is_same<TA, float>::value) {
          const f32x4_t f = ld16<f32x4_t>(vals + k4);
          v4[u][0] = f.x; v4[u][1] = f.y; v4[u][2] = f.z; v4[u][3] = f.w;
        } else if constexpr (std::is_same<TA, double>::value) {
          const f64x2_t f0 = ld16<f64x2_t>(vals + k4);
          const f64x2_t f1 = ld16<f64x2_t>(vals + k4 + 2);
          v4[u][0] = f0.x; v4[u][1] = f0.y; v4[u][2] = f1.x; v4[u][3] = f1.y;
        } else {
          const u32x4_t h = ld16<u32x4_t>(vals + k4);
          if constexpr (std::is_same<TA, HiW>::value) {
            v4[u][0] = hi_value(h.x); v4[u][1] = hi_value(h.y); v4[u][2] = hi_value(h.z); v4[u][3] = hi_value(h.w);
          } else {
            const u32x4_t lo = ld16<u32x4_t>(a.alo + k4);
            v4[u][0] = hilo_value(h.x, lo.x); v4[u][1] = hilo_value(h.y, lo.y);
            v4[u][2] = hilo_value(h.z, lo.z); v4[u][3] = hilo_value(h.w, lo.w);
          }
        }
      }
      // every gather first (the entries outside the block's range, and the
      // zero pad, hold valid column indices), so they are in flight together
      ACC xv[kU][4];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        xv[u][0] = (ACC)ldv(x[c4[u].x]);
        xv[u][1] = (ACC)ldv(x[c4[u].y]);
        xv[u][2] = (ACC)ldv(x[c4[u].z]);
        xv[u][3] = (ACC)ldv(x[c4[u].w]);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = base + u * 4 * kBlock + e;
          if (k >= p0 && k < p1) prod[k - p0] = v4[u][e] * xv[u][e];
        }
      }
    }
    __syncthreads();
    // groups of tpr lanes, tpr = the widest canonical row of the block; lanes
    // past a row's own T hold zero, which the first butterfly steps add
    for (int r = r0 + g; r < r1; r += ng) {
      ACC acc = (ACC)0;
      const int b = r == r0 + g ? rb_ : a.rp[r], e = r == r0 + g ? re_ : a.rp[r + 1];
      const int T = row_lanes(e - b);
      if (l < T)
        for (int k = b + l; k < e; k += T) acc += prod[k - p0];
      for (int o = tpr >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (l == 0) emit(r, acc);
    }
  }
  if (MODE == SM_RESID_PLAIN) {
    zsq = block_sum(zsq);
    if (t == 0) a.part[blk] = zsq;
  }
}

// Sliced ELL (64 rows per slice, one row per lane, entry k of the slice's
// rows contiguous so every load of a wave is coalesced), for matrices whose
// rows all have fewer than 2 kRowLanePer entries: their canonical sum is the
// plain sum of the rounded products in storage order, which this kernel
// keeps (no fused multiply-add), so it gives the row-block kernel's bits.
// D16: the columns are stored as 16-bit offsets from the row (column r + d),
// half the index bytes, when every entry of the matrix is within 32767 of
// its row (banded and stencil matrices).  Such a block then stages the part
// of x around its own rows, [r0 - kSellHalo, r0 + 256 + kSellHalo), in LDS
// with coalesced loads and reads the entries that fall in it from there
// (a stencil's near neighbours: one global gather each otherwise); only the
// far entries are gathered from memory.  The values summed are the same.
constexpr int kSellHalo = 128;

// The per-step finaliser of step j, run by the first n blocks of a sliced
// product launch (n = 0: none; else a multiple of 8, so the product's blocks
// keep their XCD placement): block s < S finalises system s.
struct FinArgs {
  int n = 0, j = -1;
  const double* src = nullptr;
  int rows = 0;
  const int32_t* r0 = nullptr;
  const int32_t* nr = nullptr;
};
__device__ void fin_step_block(const KArgs& a, const double* src, int rows, const int32_t* r0, const int32_t* nr,
                               int j, int s);

template <typename TA, typename TX, typename TY, int MODE, bool D16>
__global__ __launch_bounds__(kBlock) void k_sell(KArgs a, const TA* __restrict__ vals, const TX* __restrict__ x,
                                                 TY* __restrict__ y, int j, FinArgs fa) {
#pragma clang fp contract(off)
  using ACC = AccFor<TA, TY>;
  if ((int)blockIdx.x < fa.n) {
    if ((int)blockIdx.x < a.S) fin_step_block(a, fa.src, fa.rows, fa.r0, fa.nr, fa.j, blockIdx.x);
    return;
  }
  const int blk = remap_block(blockIdx.x - fa.n, gridDim.x - fa.n, a.xcd_remap);
  const int lane = threadIdx.x & 63;
  const int slice = blk * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t r = (int64_t)slice * 64 + lane;
  // the slice's extent, the row's length, the system's gate and the column
  // scale are independent loads: issue them together, before the gate test
  // (a block covers one 256-row tile of one system)
  const int on0 = gate0(a);
  const int s = a.S == 1 ? 0 : a.tile_sys[blk];
  const int off = a.sell_off[slice];
  const int w = (a.sell_off[slice + 1] - off) >> 6;
  const int len = a.sell_len[r];
  ACC scale = (ACC)1;
  if (MODE == SM_ARNOLDI && !a.wsc_defer) scale = (ACC)a.sc[(int64_t)s * (a.m + 1) + j];
  if (!gated_now(a, s, on0, off)) return;
  constexpr int kWin = D16 ? kBlock + 2 * kSellHalo : 1;
  __shared__ TX xw[kWin];
  const int64_t r0 = (int64_t)blk * kBlock;  // the block's first row
  // a slice is at most 7 entries wide (the copy is built only for rows of
  // fewer than 8), so one group of 8 covers it (entries past w are masked)
  static_assert(2 * kRowLanePer == 8, "one group of 8 entries per row");
  ACC av[8];
  int cv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int p = off + e * 64 + lane;
    av[e] = e < w ? (ACC)vals[p] : (ACC)0;
    if constexpr (D16)
      cv[e] = e < w ? (int)a.sell_dcol[p] : 0;  // offset from the row
    else
      cv[e] = e < w ? a.sell_col[p] : 0;
  }
  // the gathers go out together (a pad entry's column is its own row)
  ACC xv[8];
  if constexpr (D16) {
    // rows [r0 - halo, r0 + 256 + halo) of x, zero outside [0, ld)
    TX xl[kWin / kBlock];
#pragma unroll
    for (int q = 0; q < kWin / kBlock; ++q) {
      const int64_t c = r0 - kSellHalo + q * kBlock + threadIdx.x;
      xl[q] = (c >= 0 && c < a.ld) ? x[c] : TX{};
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int d = cv[e];
      if (d < -kSellHalo || d > kSellHalo) xv[e] = (ACC)ldv(x[(int)r + d]);
    }
#pragma unroll
    for (int q = 0; q < kWin / kBlock; ++q) xw[q * kBlock + threadIdx.x] = xl[q];
    __syncthreads();
    const int base = (int)(r - r0) + kSellHalo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int d = cv[e];
      if (d >= -kSellHalo && d <= kSellHalo) xv[e] = (ACC)ldv(xw[base + d]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[e] = (ACC)ldv(x[cv[e]]);
  }
  ACC acc = (ACC)0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if (e < len) {
      const ACC prod = av[e] * xv[e];
      acc = acc + prod;
    }
  }
  st_nt(&y[r], (TY)(acc * scale));
}

// (sc: 32-bit columns, or sd: 16-bit offsets from the row; the other is
// null.  sl: each row's length.)
__global__ void k_build_sell(KArgs a, const void* __restrict__ vals, int v32, void* __restrict__ sv,
                             int32_t* __restrict__ sc, int16_t* __restrict__ sd, uint8_t* __restrict__ sl) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.ld) return;
  const int slice = (int)(r >> 6), lane = (int)(r & 63);
  const int off = a.sell_off[slice], w = (a.sell_off[slice + 1] - off) >> 6;
  const int p0 = a.rp[r], len = a.rp[r + 1] - p0;
  sl[r] = (uint8_t)len;
  for (int k = 0; k < w; ++k) {
    const int p = off + k * 64 + lane;
    if (v32)
      static_cast<float*>(sv)[p] = k < len ? static_cast<const float*>(vals)[p0 + k] : 0.0f;
    else
      static_cast<double*>(sv)[p] = k < len ? static_cast<const double*>(vals)[p0 + k] : 0.0;
    if (sd)
      sd[p] = k < len ? (int16_t)(a.ci[p0 + k] - r) : (int16_t)0;
    else
      sc[p] = k < len ? a.ci[p0 + k] : (int32_t)r;
  }
}

// ||z||^2 and max|z| of the float64 restart residual per 256-row tile (a
// fixed tree per tile, so the norm does not depend on the row blocks).
__global__ __launch_bounds__(kBlock) void k_tile_norm(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  const SysState& S = a.st[s];
  if (S.status != RUNNING && !S.force) return;
  const double z = a.zres[(int64_t)blockIdx.x * kTile + threadIdx.x];
  const double sq = block_sum(z * z);
  const double mx = block_max(fabs(z));
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = sq;
    a.part[(int64_t)a.ntile + blockIdx.x] = mx;
  }
}

// ------------------------------------------------------- buffer loads
// The basis is read through one buffer resource: a per-lane byte offset of
// the row plus a scalar byte offset of the column, so a register tile of up
// to 64 columns needs no per-column 64-bit addresses.  Reads past the end
// of the resource return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
template <>
__device__ __forceinline__ bf16_t bload<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return bf16_t{(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0)};
}
template <>
__device__ __forceinline__ f16_t bload<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f16_t, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
}
// The same loads with the non-temporal hint (cache policy bit 1 on gfx950):
// rows of a CGSR pass that the memory-side cache could not keep until the
// next pass reaches them, so they need not displace the rows it can keep.
template <typename T>
__device__ __forceinline__ T bload_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff);
template <>
__device__ __forceinline__ float bload_nt<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 2));
}
template <>
__device__ __forceinline__ double bload_nt<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, 2);
  return __hiloint2double((int)v[1], (int)v[0]);
}
template <>
__device__ __forceinline__ bf16_t bload_nt<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return bf16_t{(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, 0, 2)};
}
template <>
__device__ __forceinline__ f16_t bload_nt<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(f16_t, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, 0, 2));
}
// Memory-side cache policy of the CGSR passes.  Each workgroup walks its own
// tile range, and the next pass over the basis walks it the other way, so
// only the last tiles a pass touches are still cached when the next pass
// starts.  A pass over B bytes of basis keeps (with ordinary loads) the last
// keep / B of every range; the tiles before them would be evicted before the
// next pass reaches them, so they are read non-temporally.  The two
// projections keep kMallKeep; the last pass keeps less (kMallKeepLast), for
// the next step's projection 1, because the Arnoldi product between them
// streams A and does better when part of A is still cached from the step
// before (measured on the 128^3 stencil: 192 MB there made the product 7 %
// slower, 48 MB made it 1 % faster, and saved 1.8 ms of projection 1 per
// solve).
constexpr uint64_t kMallKeep = 192ull << 20;
constexpr uint64_t kMallKeepLast = 48ull << 20;

// (2-byte bases: never split, which keeps their 64-column tile free of
// spills under the 128-register cap.)
template <typename TV>
__device__ __forceinline__ int nt_tiles(int nt, uint64_t pass_bytes, uint64_t keep = kMallKeep) {
  if (sizeof(TV) == 2 || pass_bytes <= keep) return 0;
  return nt - (int)(((uint64_t)nt * keep + pass_bytes - 1) / pass_bytes);
}

// A register tile of L basis columns [col0, col0 + L) is read through two
// resources, one per half: half h starts at column col0 + h L/2 and is
// bounded to the columns below col0 + ncol, so columns past ncol read zero
// with no per-column guard, and column q's offset within its half is the
// plain (q mod L/2) * cs (below L/2 columns, which the create-time size
// check keeps inside 32 bits).
struct TileRsrc {
  __amdgpu_buffer_rsrc_t half[2];
};
template <typename TV, int L>
__device__ __forceinline__ TileRsrc tile_rsrc(const KArgs& a, int col0, int ncol) {
  constexpr int H = L / 2;
  const int64_t cb = a.ld * (int64_t)sizeof(TV);
  const TV* base = reinterpret_cast<const TV*>(a.V) + (int64_t)col0 * a.ld;
  TileRsrc t;
  t.half[0] = make_rsrc(base, (uint32_t)((int64_t)min(ncol, H) * cb));
  t.half[1] = make_rsrc(base + (int64_t)H * a.ld, (uint32_t)((int64_t)max(ncol - H, 0) * cb));
  return t;
}

// One tile of basis loads: column q at byte offset voff + (q mod L/2) * cs
// of its half's resource.
template <typename TV, int L, bool kNT, typename ACC>
__device__ __forceinline__ void load_tile(ACC (&v)[L], const TileRsrc& rs, uint32_t voff, uint32_t cs) {
  constexpr int H = L / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t so = 0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      v[h * H + q] = (ACC)ldv(kNT ? bload_nt<TV>(rs.half[h], voff + so) : bload<TV>(rs.half[h], voff + so, 0));
      so += cs;
    }
  }
}


// ------------------------------------------------------- persistent passes

// Logical workgroup of a persistent pass: consecutive logical workgroups are
// placed on one XCD, and passes that re-read the same basis columns alternate
// direction so each starts on the rows the previous pass touched last, which
// the memory-side cache still holds.
__device__ __forceinline__ int pass_block(const KArgs& a, const SegTab& sg, int rev) {
  const int b = remap_block(blockIdx.x, sg.G, a.xcd_remap);
  return rev ? sg.G - 1 - b : b;
}

// Row of tile u of a segment (first tile t0, nt tiles) for this thread; the
// passes read t0 and nt once before their tile loop (a loop that re-read
// them would wait for that load before every tile's addresses).
__device__ __forceinline__ int64_t seg_row(int t0, int nt, int u, int rev) {
  const int tile = rev ? t0 + nt - 1 - u : t0 + u;
  return (int64_t)tile * kTile + threadIdx.x;
}

// Segments of a pass without table reads where they are known: with one
// system every segment is system 0's, and when its tiles cover every
// workgroup (nseg = G) workgroup b holds exactly segment b, tiles
// [b T / G, (b + 1) T / G).  Passes start with these instead of dependent
// loads of the split tables (which the streamed basis evicts from L2
// between launches), and test the single system's gate, loaded at the
// kernel's start, instead of loading it per segment.
__device__ __forceinline__ bool seg_direct(const KArgs& a, const SegTab& sg) {
  return a.S == 1 && sg.nseg == sg.G;
}
__device__ __forceinline__ int seg_k0(const KArgs& a, const SegTab& sg, int b) {
  return seg_direct(a, sg) ? b : sg.bseg0[b];
}
__device__ __forceinline__ int seg_k1(const KArgs& a, const SegTab& sg, int b) {
  return seg_direct(a, sg) ? b + 1 : sg.bseg0[b + 1];
}
__device__ __forceinline__ int seg_sys(const KArgs& a, const SegTab& sg, int k) {
  return a.S == 1 ? 0 : sg.seg_sys[k];
}
__device__ __forceinline__ void seg_tiles(const KArgs& a, const SegTab& sg, int k, int& t0, int& nt) {
  if (seg_direct(a, sg)) {
    t0 = (int)((int64_t)k * a.ntile / sg.G);
    nt = (int)((int64_t)(k + 1) * a.ntile / sg.G) - t0;
  } else {
    t0 = sg.seg_t0[k];
    nt = sg.seg_nt[k];
  }
}
__device__ __forceinline__ int sys_seg0(const KArgs& a, const SegTab& sg, int s) {
  return a.S == 1 ? 0 : sg.sys_sg0[s];
}
__device__ __forceinline__ int sys_nseg(const KArgs& a, const SegTab& sg, int s) {
  return a.S == 1 ? sg.nseg : sg.sys_nsg[s];
}
// gate of system s, with on0 = gate0() for a single system
__device__ __forceinline__ bool gated_s(const KArgs& a, int s, int on0) {
  return a.S == 1 ? on0 != 0 : gated(a, s);
}

template <typename T>
__device__ __forceinline__ const T* col_ptr(const KArgs& a, int i) {
  return reinterpret_cast<const T*>(a.V) + (int64_t)i * a.ld;
}

// Per-wave column sums (lane-owned after reduce_scatter) to quantities
// col0 .. col0 + ncol - 1 of partial row k, in a fixed cross-wave order.
template <int L, typename ACC>
__device__ __forceinline__ void store_colsums(double* part, int nrows, int k, int col0, int ncol,
                                              ACC colsum) {
  __shared__ ACC lds[kBlock / 64][L];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int R = 64 / L;  // lanes per column
  if ((lane & (R - 1)) == 0) lds[wv][lane / R] = colsum;
  __syncthreads();
  if (threadIdx.x < ncol) {
    ACC tot = lds[0][threadIdx.x];
#pragma unroll
    for (int q = 1; q < kBlock / 64; ++q) tot += lds[q][threadIdx.x];
    part[(int64_t)(col0 + threadIdx.x) * nrows + k] = (double)tot;
  }
  __syncthreads();
}

// CGSR projection, first half: quantities col0 .. of V^T w for the columns
// [col0, col0 + L) below j + 1, plus ||w||^2 (quantity j + 1) when col0 = 0
// and mode = 1.  mode 2: the second projection's dots when j + 1 > 64.
// mode 3: the loss-of-orthogonality monitor's dots, with basis column j + 1
// (as stored, before its decode scale) in place of w.
//
// DS (the k_mdot_ds variant, 4- and 8-byte bases): projection 1 also applies
// v_j's decode scale to w, which the Arnoldi product left out (wsc_defer).
template <typename TV, typename TW, int L, bool DS>
__device__ __forceinline__ void mdot_body(const KArgs& a, const SegTab& sg, int j, int col0, int mode, int rev) {
  using ACC = AccFor<TV, TW>;
  const int b = pass_block(a, sg, rev);
  const int lane = threadIdx.x & 63;
  const int ncol = min(L, j + 1 - col0);
  const TW* w = reinterpret_cast<const TW*>(a.w);
  const TV* wv = reinterpret_cast<const TV*>(a.V) + (int64_t)(j + 1) * a.ld;
  const TileRsrc rs = tile_rsrc<TV, L>(a, col0, ncol);
  const uint32_t cstride = (uint32_t)(a.ld * (int64_t)sizeof(TV));
  uint32_t cs = cstride;
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    // projection 1 applies v_j's decode scale to w when the product left it
    // out: the product's own rounding, kept apart from the sums that follow
    const bool defer = DS && mode == 1;
    const ACC wsc = defer ? (ACC)a.sc[(int64_t)s * (a.m + 1) + j] : (ACC)1;
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    const int nfirst = nt_tiles<TV>(nt, (uint64_t)ncol * (uint64_t)cstride);
    ACC colsum = (ACC)0, ww = (ACC)0;
    // narrow tiles move few bytes per load round: UT of them per iteration
    // keep as many loads in flight as a wider tile (sums stay tile by tile)
    constexpr int UT = L <= 16 ? 2 : 1;
#pragma unroll 1
    for (int u = 0; u < nt; u += UT) {
      // column offsets are rebuilt per tile (a scalar add each) instead of
      // being hoisted into L/2 live scalar registers
      asm volatile("" : "+s"(cs));
      ACC p[UT][L], wr[UT];
#pragma unroll
      for (int h = 0; h < UT; ++h) {
        const int uu = u + h < nt ? u + h : u;
        const int64_t r = seg_row(t0, nt, uu, rev);
        const uint32_t voff = (uint32_t)(r * (int64_t)sizeof(TV));
        wr[h] = mode == 3 ? (ACC)ldv(wv[r]) : (ACC)w[r];
        if (defer) wr[h] = mul_nofuse(wr[h], wsc);
        if (sizeof(TV) != 2 && uu < nfirst)
          load_tile<TV, L, true>(p[h], rs, voff, cs);
        else
          load_tile<TV, L, false>(p[h], rs, voff, cs);
      }
#pragma unroll
      for (int h = 0; h < UT; ++h) {
        if (u + h >= nt) break;
        ww += wr[h] * wr[h];
#pragma unroll
        for (int q = 0; q < L; ++q) p[h][q] *= wr[h];
        colsum += reduce_scatter<L>(p[h], lane);
      }
    }
    store_colsums<L>(a.part, sg.nseg, k, col0, ncol, colsum);
    if (col0 == 0 && mode == 1) {
      const ACC tot = block_sum(ww);
      if (threadIdx.x == 0) a.part[(int64_t)(j + 1) * sg.nseg + k] = (double)tot;
    }
  }
}
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_mdot(KArgs a, SegTab sg, int j, int col0, int mode, int rev) {
  mdot_body<TV, TW, L, false>(a, sg, j, col0, mode, rev);
}
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_mdot_ds(KArgs a, SegTab sg, int j, int col0, int mode, int rev) {
  mdot_body<TV, TW, L, true>(a, sg, j, col0, mode, rev);
}

// CGSR projection 2, fused: w' = w - V coef (coef from projection 1), then
// V^T w' from the same register tile of V.  Requires j + 1 <= L <= 64.  DS
// (the _ds kernels): w is first scaled by v_j's decode scale, as in
// projection 1.
template <typename TV, typename TW, int L, bool DS>
__device__ __forceinline__ void axpy_mdot_body(const KArgs& a, const SegTab& sg, int j, int rev) {
  using ACC = AccFor<TV, TW>;
  const int b = pass_block(a, sg, rev);
  const int t = threadIdx.x, lane = t & 63;
  const int ncol = j + 1;
  TW* w = reinterpret_cast<TW*>(a.w);
  const TileRsrc rs = tile_rsrc<TV, L>(a, 0, ncol);
  const uint32_t cstride = (uint32_t)(a.ld * (int64_t)sizeof(TV));
  uint32_t cs = cstride;
  __shared__ ACC cf[L];
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const double* coefd = a.coef + (int64_t)s * (a.m + 2);
    if (t < L) cf[t] = (t < ncol) ? (ACC)coefd[t] : (ACC)0;
    // (the decode scale of v_j, when the product left it out of w)
    const ACC wsc = DS ? (ACC)a.sc[(int64_t)s * (a.m + 1) + j] : (ACC)1;
    __syncthreads();
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    const int nfirst = nt_tiles<TV>(nt, (uint64_t)ncol * (uint64_t)cstride);
    ACC colsum = (ACC)0;
#pragma unroll 1
    for (int u = 0; u < nt; ++u) {
      asm volatile("" : "+s"(cs));
      const int64_t r = seg_row(t0, nt, u, rev);
      const uint32_t voff = (uint32_t)(r * (int64_t)sizeof(TV));
      ACC v[L];
      if (sizeof(TV) != 2 && u < nfirst)
        load_tile<TV, L, true>(v, rs, voff, cs);
      else
        load_tile<TV, L, false>(v, rs, voff, cs);
      ACC wr = (ACC)w[r];
      if (DS) wr = mul_nofuse(wr, wsc);  // (the product's rounding, as above)
#pragma unroll
      for (int q = 0; q < L; ++q) wr -= cf[q] * v[q];
      st_nt(&w[r], (TW)wr);
#pragma unroll
      for (int q = 0; q < L; ++q) v[q] *= wr;
      colsum += reduce_scatter<L>(v, lane);
    }
    store_colsums<L>(a.part, sg.nseg, k, 0, ncol, colsum);
  }
}

// float32 w (4-byte and 2-byte bases): capped at 128 registers so four
// workgroups fit on a CU; with float64 w the tile is held in float64 and
// needs more registers than that (k_axpy_mdot64).
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_axpy_mdot(KArgs a, SegTab sg, int j, int rev) {
  axpy_mdot_body<TV, TW, L, false>(a, sg, j, rev);
}
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_axpy_mdot_ds(KArgs a, SegTab sg, int j, int rev) {
  axpy_mdot_body<TV, TW, L, true>(a, sg, j, rev);
}
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_axpy_mdot64(KArgs a, SegTab sg, int j, int rev) {
  axpy_mdot_body<TV, TW, L, false>(a, sg, j, rev);
}
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_axpy_mdot64_ds(KArgs a, SegTab sg, int j, int rev) {
  axpy_mdot_body<TV, TW, L, true>(a, sg, j, rev);
}

// w -= V[:, col0:col0+L] coef (no reduction): the first half of projection 2
// when j + 1 > 64.
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_axpy(KArgs a, SegTab sg, int j, int col0) {
  using ACC = AccFor<TV, TW>;
  const int b = pass_block(a, sg, 0);
  const int ncol = min(L, j + 1 - col0);
  TW* w = reinterpret_cast<TW*>(a.w);
  const TV* V0 = col_ptr<TV>(a, col0);
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const double* coefd = a.coef + (int64_t)s * (a.m + 2) + col0;
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    for (int u = 0; u < nt; ++u) {
      const int64_t r = seg_row(t0, nt, u, 0);
      ACC wr = (ACC)w[r];
      for (int q = 0; q < ncol; ++q) wr -= (ACC)coefd[q] * (ACC)ldv(V0[(int64_t)q * a.ld + r]);
      st_nt(&w[r], (TW)wr);
    }
  }
}

// Writes the end-of-step partials (||w''||^2, max|w''|) of segment k.
template <typename ACC>
__device__ __forceinline__ void store_norm_partials(double* part, int nrows, int k, ACC sq, ACC mx) {
  const double tsq = (double)block_sum(sq);
  const double tmx = (double)block_max(mx);
  if (threadIdx.x == 0) {
    part[k] = tsq;
    part[(int64_t)nrows + k] = tmx;
  }
}

// Last CGSR pass of a step: w'' = w' - sum_{i <= j} coef_i v_i with the whole
// tile of basis loads in flight (j + 1 <= L <= 64), ||w''||^2 and max|w''|.
// w'' goes to basis column j+1 (float32 / float64 basis, normalised by the
// decode scale 1/h_{j+1,j}) or stays in w (2-byte basis, encoded later).
template <typename TV, typename TW, int L>
__global__ __launch_bounds__(kBlock) void k_final_tile(KArgs a, SegTab sg, int j, int rev) {
  using ACC = AccFor<TV, TW>;
  constexpr bool kTwoByte = sizeof(TV) == 2;
  const int b = pass_block(a, sg, rev);
  const int t = threadIdx.x;
  const int ncol = j + 1;
  TW* w = reinterpret_cast<TW*>(a.w);
  const TileRsrc rs = tile_rsrc<TV, L>(a, 0, ncol);
  const uint32_t cstride = (uint32_t)(a.ld * (int64_t)sizeof(TV));
  uint32_t cs = cstride;
  TV* vout = reinterpret_cast<TV*>(a.V) + (int64_t)(j + 1) * a.ld;
  __shared__ ACC cf[L];
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const double* coefd = a.coef + (int64_t)s * (a.m + 2);
    if (t < L) cf[t] = (t < ncol) ? (ACC)coefd[t] : (ACC)0;
    __syncthreads();
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    const int nfirst = nt_tiles<TV>(nt, (uint64_t)ncol * (uint64_t)cstride, kMallKeepLast);
    ACC sq = (ACC)0, mx = (ACC)0;
#pragma unroll 1
    for (int u = 0; u < nt; ++u) {
      asm volatile("" : "+s"(cs));
      const int64_t r = seg_row(t0, nt, u, rev);
      const uint32_t voff = (uint32_t)(r * (int64_t)sizeof(TV));
      ACC v[L];
      if (sizeof(TV) == 2 || u < nfirst)
        load_tile<TV, L, true>(v, rs, voff, cs);
      else
        load_tile<TV, L, false>(v, rs, voff, cs);
      ACC wr = (ACC)w[r];
#pragma unroll
      for (int q = 0; q < L; ++q) wr -= cf[q] * v[q];
      sq += wr * wr;
      mx = fmax(mx, fabs(wr));
      if constexpr (kTwoByte)
        st_nt(&w[r], (TW)wr);
      else
        st_nt(&vout[r], (TV)wr);
    }
    store_norm_partials(a.part, sg.nseg, k, sq, mx);
  }
}

// The same last pass for j + 1 > 64 (column loop instead of a register tile).
template <typename TV, typename TW>
__global__ __launch_bounds__(kBlock) void k_final(KArgs a, SegTab sg, int j) {
  using ACC = AccFor<TV, TW>;
  constexpr bool kTwoByte = sizeof(TV) == 2;
  const int b = pass_block(a, sg, 0);
  TW* w = reinterpret_cast<TW*>(a.w);
  TV* vout = reinterpret_cast<TV*>(a.V) + (int64_t)(j + 1) * a.ld;
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const double* coefd = a.coef + (int64_t)s * (a.m + 2);
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    ACC sq = (ACC)0, mx = (ACC)0;
    for (int u = 0; u < nt; ++u) {
      const int64_t r = seg_row(t0, nt, u, 0);
      ACC wr = (ACC)w[r];
      for (int i = 0; i <= j; ++i) wr -= (ACC)coefd[i] * (ACC)ldv(col_ptr<TV>(a, i)[r]);
      sq += wr * wr;
      mx = fmax(mx, fabs(wr));
      if constexpr (kTwoByte)
        st_nt(&w[r], (TW)wr);
      else
        st_nt(&vout[r], (TV)wr);
    }
    store_norm_partials(a.part, sg.nseg, k, sq, mx);
  }
}

// MGS, fused: step i of Arnoldi column j first completes dot i-1 itself
// (every workgroup reduces the previous launch's partials of its system in
// the same fixed order, so all hold the same h_{i-1}; the workgroup owning
// the system's first segment records it in H), then w -= h_{i-1} v_{i-1} and
// the partial dot w . v_i.  Partial tables alternate by the parity of i.
constexpr int kMgsUnroll = 4;
// the MGS steps use a fixed grid of kMgsOcc workgroups per CU: a step is
// short, so the partial rows every workgroup re-reduces are kept few
constexpr int kMgsOcc = 4;

__device__ __forceinline__ double mgs_complete(const KArgs& a, const SegTab& sgp, int s, bool first,
                                               int i, const double* pin) {
  const int g0 = sys_seg0(a, sgp, s), ng = sys_nseg(a, sgp, s);
  const int M1 = a.m + 1, M2 = a.m + 2;
  const double d = reduce_col<false>(pin + g0, ng);
  const double sci = a.sc[(int64_t)s * M1 + i];
  const double h = sci * d;
  if (first) {
    double wn = 0.0;
    if (i == 0) wn = sqrt(reduce_col<false>(pin + sgp.nseg + g0, ng));
    if (threadIdx.x == 0) {
      a.hacc[(int64_t)s * M2 + i] = h;
      a.coef[(int64_t)s * M2 + i] = h * sci;
      if (i == 0) a.st[s].wnorm_pre = wn;
    }
  }
  return h * sci;
}

template <typename TV, typename TW>
__global__ __launch_bounds__(kBlock) void k_mgs(KArgs a, SegTab sg, int j, int i) {
  using ACC = AccFor<TV, TW>;
  const int b = pass_block(a, sg, i & 1);
  double* pout = (i & 1) ? a.part2 : a.part;
  const double* pin = (i & 1) ? a.part : a.part2;  // dot i-1
  TW* w = reinterpret_cast<TW*>(a.w);
  const TV* vi = col_ptr<TV>(a, i);
  const TV* vp = col_ptr<TV>(a, i > 0 ? i - 1 : 0);
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const ACC cprev = i > 0 ? (ACC)mgs_complete(a, sg, s, k == sys_seg0(a, sg, s), i - 1, pin) : (ACC)0;
    // steps 0 and 1 read w as the Arnoldi product stored it: without v_j's
    // decode scale when the product left it out (applied here with the
    // product's rounding, apart from the sums that follow)
    const bool ds = a.wsc_defer && i <= 1;
    const ACC wsc = ds ? (ACC)a.sc[(int64_t)s * (a.m + 1) + j] : (ACC)1;
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    ACC d = (ACC)0, ww = (ACC)0;
    // kMgsUnroll tiles per iteration: all their loads are issued before use
    for (int u = 0; u < nt; u += kMgsUnroll) {
      int64_t r[kMgsUnroll];
      ACC wv[kMgsUnroll], pv[kMgsUnroll], iv[kMgsUnroll];
#pragma unroll
      for (int q = 0; q < kMgsUnroll; ++q) {
        r[q] = seg_row(t0, nt, u + q < nt ? u + q : u, i & 1);
        wv[q] = (ACC)w[r[q]];
        if (ds) wv[q] = mul_nofuse(wv[q], wsc);
        pv[q] = i > 0 ? (ACC)ldv(vp[r[q]]) : (ACC)0;
        iv[q] = (ACC)ldv(vi[r[q]]);
      }
#pragma unroll
      for (int q = 0; q < kMgsUnroll; ++q) {
        if (u + q >= nt) continue;
        ACC wr = wv[q];
        if (i > 0) {
          wr -= cprev * pv[q];
          st_nt(&w[r[q]], (TW)wr);
        } else {
          ww += wr * wr;
        }
        d += wr * iv[q];
      }
    }
    const double td = (double)block_sum(d);
    double tw = 0.0;
    if (i == 0) tw = (double)block_sum(ww);
    if (threadIdx.x == 0) {
      pout[k] = td;
      if (i == 0) pout[(int64_t)sg.nseg + k] = tw;
    }
  }
}

// Last MGS pass of column j: completes dot j (partials written by k_mgs with
// split sgp), w'' = w - h_j v_j, and the partials of ||w''||^2, max|w''|.
template <typename TV, typename TW>
__global__ __launch_bounds__(kBlock) void k_mgs_final(KArgs a, SegTab sg, SegTab sgp, int j) {
  using ACC = AccFor<TV, TW>;
  constexpr bool kTwoByte = sizeof(TV) == 2;
  const int b = pass_block(a, sg, (j + 1) & 1);
  const double* pin = (j & 1) ? a.part2 : a.part;
  double* pout = (j & 1) ? a.part : a.part2;
  TW* w = reinterpret_cast<TW*>(a.w);
  const TV* vj = col_ptr<TV>(a, j);
  TV* vout = reinterpret_cast<TV*>(a.V) + (int64_t)(j + 1) * a.ld;
  const int on0 = gate0(a);
  for (int k = seg_k0(a, sg, b), k1 = seg_k1(a, sg, b); k < k1; ++k) {
    const int s = seg_sys(a, sg, k);
    if (!gated_s(a, s, on0)) continue;
    const ACC cj = (ACC)mgs_complete(a, sgp, s, k == sys_seg0(a, sg, s), j, pin);
    // (at j = 0 no step has stored w yet: the deferred scale, as in k_mgs)
    const bool ds = a.wsc_defer && j == 0;
    const ACC wsc = ds ? (ACC)a.sc[(int64_t)s * (a.m + 1) + j] : (ACC)1;
    int t0, nt;
    seg_tiles(a, sg, k, t0, nt);
    ACC sq = (ACC)0, mx = (ACC)0;
    for (int u = 0; u < nt; u += kMgsUnroll) {
      int64_t r[kMgsUnroll];
      ACC wv[kMgsUnroll], jv[kMgsUnroll];
#pragma unroll
      for (int q = 0; q < kMgsUnroll; ++q) {
        r[q] = seg_row(t0, nt, u + q < nt ? u + q : u, (j + 1) & 1);
        wv[q] = (ACC)w[r[q]];
        if (ds) wv[q] = mul_nofuse(wv[q], wsc);
        jv[q] = (ACC)ldv(vj[r[q]]);
      }
#pragma unroll
      for (int q = 0; q < kMgsUnroll; ++q) {
        if (u + q >= nt) continue;
        const ACC wr = wv[q] - cj * jv[q];
        sq += wr * wr;
        mx = fmax(mx, fabs(wr));
        if constexpr (kTwoByte)
          st_nt(&w[r[q]], (TW)wr);
        else
          st_nt(&vout[r[q]], (TV)wr);
      }
    }
    store_norm_partials(pout, sg.nseg, k, sq, mx);
  }
}

// ---------------------------------------------------------------- finalise
// The per-system completions read the partial rows the preceding pass wrote
// (the kernel boundary makes them visible) and run the system's scalar step.

enum FinMode { FIN_STEP = 0, FIN_RESID = 1, FIN_BNORM = 2, FIN_LEFT = 3, FIN_BNORMP = 4 };

// Left preconditioning, at the start of a cycle: beta = ||M^-1 z|| becomes
// s_1 and the reference of the improvement trigger, and v_1 = M^-1 z / beta
// gets its decode scale.  A zero or non-finite M^-1 z switches the
// preconditioner off and ends the cycle without a correction (the next one
// runs plain GMRES from the same x).
__device__ void fin_left(const KArgs& a, int s, double sumsq, double wmax) {
  SysState& S = a.st[s];
  const int M1 = a.m + 1;
  const double beta = sqrt(sumsq);
  if (!(beta > 0.0) || !isfinite(beta)) {
    S.active = 0;
    S.precond_on = 0;
    S.fallback_used = 1;
    return;
  }
  S.beta = beta;
  a.s[(int64_t)s * M1] = beta;
  a.ares[(int64_t)s * M1] = beta;
  if (a.prec == PBF16 || a.prec == PF16) {
    const int e = scale_exp(wmax / beta, a.prec);
    a.sc[(int64_t)s * M1] = ldexp(1.0, -e);
    S.enc_f = (float)(ldexp(1.0, e) / beta);
  } else {
    a.sc[(int64_t)s * M1] = 1.0 / beta;
  }
}

// `src` with column stride `rows`; system s owns rows [r0[s], r0[s] + nr[s]).
template <int MODE>
__global__ __launch_bounds__(kFinBlock) void k_fin(KArgs a, const double* src, int rows, const int32_t* r0,
                                                  const int32_t* nr, int j) {
  const int s = blockIdx.x;
  const SysState& S = a.st[s];
  if (MODE == FIN_RESID) {
    if (S.status != RUNNING && !S.force) return;
  } else if (MODE == FIN_STEP) {
    if (!S.active && !S.force) return;
  } else if (MODE == FIN_LEFT) {
    if (!S.active || !S.precond_on) return;
  }
  const int b0 = r0[s], n = nr[s];
  const double sq = reduce_col<false>(src + b0, n);
  if (MODE == FIN_BNORM || MODE == FIN_BNORMP) {
    if (threadIdx.x == 0) {
      SysState& W = a.st[s];
      if (MODE == FIN_BNORMP) {
        W.bnorm_p = sqrt(sq);
        return;
      }
      W.bnorm = sqrt(sq);
      W.bnorm_p = W.bnorm;
      if (W.bnorm == 0.0) {
        W.status = CONVERGED;
        W.rel = 0.0;
      }
    }
    return;
  }
  const double mx = reduce_col<true>(src + rows + b0, n);
  if (threadIdx.x == 0) {
    if (MODE == FIN_LEFT)
      fin_left(a, s, sq, mx);
    else
      fin_residual(a, s, sq, mx);
  }
}

// Sum of p[0, n) and maximum of q[0, n), both in a fixed order, in one pass
// (every thread of the block returns both).
__device__ void reduce_sum_max(const double* p, const double* q, int n, double& sum, double& mx) {
  __shared__ double sh[2][kBlock / 64];
  const int t = threadIdx.x, NT = blockDim.x;
  double s0 = 0.0, s1 = 0.0, m0 = 0.0, m1 = 0.0;
  int r = t;
  for (; r + NT < n; r += 2 * NT) {
    s0 += p[r];
    s1 += p[r + NT];
    m0 = fmax(m0, q[r]);
    m1 = fmax(m1, q[r + NT]);
  }
  if (r < n) {
    s0 += p[r];
    m0 = fmax(m0, q[r]);
  }
  double v = wave_sum(s0 + s1), w = wave_max(fmax(m0, m1));
  if ((t & 63) == 0) {
    sh[0][t >> 6] = v;
    sh[1][t >> 6] = w;
  }
  __syncthreads();
  sum = sh[0][0];
  mx = sh[1][0];
  for (int k = 1; k < NT / 64; ++k) {
    sum += sh[0][k];
    mx = fmax(mx, sh[1][k]);
  }
}

// The per-step finaliser: column j of H from the float64 partials of the
// last pass (||w''||^2 in the first column of src, max|w''| in the second),
// the Givens step and the restart decisions, on an LDS copy of the state.
__device__ void fin_step_block(const KArgs& a, const double* src, int rows, const int32_t* r0, const int32_t* nr,
                               int j, int s) {
  __shared__ FinShared sh;
  __shared__ SysState S;
  const int t = threadIdx.x;
  const SysState& G = a.st[s];
  // the state copy, the staged column and rotations and the partial rows are
  // loaded before the gate is tested (they do not depend on it), so they
  // take one memory round trip together
  const int on0 = gate0(a);
  constexpr int kWords = (int)(sizeof(SysState) / 8);
  static_assert(sizeof(SysState) % 8 == 0, "SysState is copied as 8-byte words");
  if (t < kWords) reinterpret_cast<uint64_t*>(&S)[t] = reinterpret_cast<const uint64_t*>(&G)[t];
  fin_stage(a, s, j, sh);
  const int b0 = a.S == 1 ? 0 : r0[s];
  const int n = a.S == 1 ? rows : nr[s];
  double sq, mx;
  reduce_sum_max(src + b0, src + rows + b0, n, sq, mx);
  if (!gated_now(a, s, on0, n)) return;
  fin_step(a, s, j, sq, mx, S, sh);
  __syncthreads();
  if (t < kWords) reinterpret_cast<uint64_t*>(&a.st[s])[t] = reinterpret_cast<const uint64_t*>(&S)[t];
}

__global__ __launch_bounds__(kBlock) void k_fin_step(KArgs a, const double* src, int rows, const int32_t* r0,
                                                     const int32_t* nr, int j) {
  fin_step_block(a, src, rows, r0, nr, j, blockIdx.x);
}

// The CGS projections complete column by column: workgroup (s, q) reduces
// quantity q of system s.  Pass 1: h1_q = sc_q * sum and the next axpy
// coefficient h1_q * sc_q (quantity j+1 carries ||w||^2).  Pass 2: h2_q, the
// column of H (h1 + h2) and the coefficient h2_q * sc_q.
// A completion is a few dependent memory round trips on one CU, so every
// load it needs (the gate, the column's scale and h1 entry, the partial
// rows) is issued before the gate is tested; a gated-off system's block
// reduces and drops the result.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_fin_cols(KArgs a, SegTab sg, int j) {
  const int s = blockIdx.x, q = blockIdx.y;
  const int M1 = a.m + 1, M2 = a.m + 2;
  const int on0 = gate0(a);
  const double scq = a.sc[(int64_t)s * M1 + q];
  const double h1q = PASS == 2 ? a.h1[(int64_t)s * M2 + q] : 0.0;
  const int g0 = sys_seg0(a, sg, s);
  const int ng = sys_nseg(a, sg, s);
  const double v = reduce_col<false>(a.part + (int64_t)q * sg.nseg + g0, ng);
  if (!gated_now(a, s, on0, ng) || threadIdx.x != 0) return;
  if (PASS == 1 && q == j + 1) {
    a.st[s].wnorm_pre = sqrt(v);
    return;
  }
  const double h = scq * v;
  if (PASS == 1)
    a.h1[(int64_t)s * M2 + q] = h;
  else
    a.hacc[(int64_t)s * M2 + q] = h1q + h;
  a.coef[(int64_t)s * M2 + q] = h * scq;
}

// Loss-of-orthogonality monitor (the last restart strategy of section 3).
// u = V_j^T v_{j+1} with the decoded columns: workgroup (s, q) reduces
// quantity q of system s.
__global__ __launch_bounds__(kBlock) void k_orth_cols(KArgs a, SegTab sg, int j) {
  const int s = blockIdx.x, q = blockIdx.y;
  const SysState& S = a.st[s];
  if (!S.active && !S.force) return;
  const double v = reduce_col<false>(a.part + (int64_t)q * sg.nseg + sys_seg0(a, sg, s), sys_nseg(a, sg, s));
  if (threadIdx.x != 0) return;
  const int M1 = a.m + 1;
  a.ocol[(int64_t)s * M1 + q] = v * a.sc[(int64_t)s * M1 + q] * a.sc[(int64_t)s * M1 + j + 1];
}

// Column c = j + 1 of U and of S = (I + U)^-1 U (S_{k+1} = [S_k, (I + U_k)^-1 u;
// 0, 0], a back-substitution with the unit upper triangular I + U_k), then
// ||S||_F (running sum) or ||S||_2 (10 power iterations on S^T S from the
// all-ones vector, then ||S x||); the cycle ends once it reaches the
// threshold.  One workgroup per system; U, then S, staged in LDS.
__global__ __launch_bounds__(kBlock) void k_orth_fin(KArgs a, int j) {
  __shared__ double mat[(kMaxOrthM + 1) * (kMaxOrthM + 1)];
  __shared__ double sv[kMaxOrthM + 2], xv[kMaxOrthM + 2], yv[kMaxOrthM + 2];
  __shared__ double red[kBlock / 64];
  const int s = blockIdx.x, t = threadIdx.x;
  SysState& S = a.st[s];
  if (!S.active && !S.force) return;
  const int M1 = a.m + 1, c = j + 1, k = j + 2;  // S is k x k; new column c
  double* OU = a.ou + (int64_t)s * M1 * M1;
  double* OS = a.os + (int64_t)s * M1 * M1;
  const double* u = a.ocol + (int64_t)s * M1;
  // U's leading c x c block (columns 1..c-1 hold data; column-major, stride M1)
  for (int i = t; i < c * c; i += kBlock) {
    const int col = i / c, row = i % c;
    mat[col * c + row] = row < col ? OU[(int64_t)col * M1 + row] : 0.0;
  }
  for (int i = t; i < c; i += kBlock) {
    sv[i] = u[i];
    OU[(int64_t)c * M1 + i] = u[i];
  }
  __syncthreads();
  if (t == 0) {  // (I + U) s = u, rows c-1 .. 0
    for (int r = c - 1; r >= 0; --r) {
      double acc = sv[r];
      for (int l = r + 1; l < c; ++l) acc -= mat[l * c + r] * sv[l];
      sv[r] = acc;
    }
  }
  __syncthreads();
  double f2 = 0.0;
  for (int i = t; i < c; i += kBlock) {
    OS[(int64_t)c * M1 + i] = sv[i];
    f2 += sv[i] * sv[i];
  }
  f2 = block_sum(f2);
  const double fro2 = (j == 0 ? 0.0 : S.orth_fro2) + f2;
  double nrm = sqrt(fro2);
  if (a.orth_norm == 0) {
    // S in LDS (k x k, column-major, zero on and below the diagonal)
    __syncthreads();
    for (int i = t; i < k * k; i += kBlock) {
      const int col = i / k, row = i % k;
      mat[col * k + row] = (row < col && col >= 1) ? (col == c ? sv[row] : OS[(int64_t)col * M1 + row]) : 0.0;
    }
    const double x0 = 1.0 / sqrt((double)k);
    for (int i = t; i < k; i += kBlock) xv[i] = x0;
    __syncthreads();
    bool zero = false;
    for (int it = 0; it < 10 && !zero; ++it) {
      for (int i = t; i < k; i += kBlock) {  // y = S x
        double acc = 0.0;
        for (int l = i + 1; l < k; ++l) acc += mat[l * k + i] * xv[l];
        yv[i] = acc;
      }
      __syncthreads();
      double z2 = 0.0;
      double zi = 0.0;
      if (t < k) {  // z = S^T y, thread t owns column t
        for (int l = 0; l < t; ++l) zi += mat[t * k + l] * yv[l];
        z2 = zi * zi;
      }
      z2 = block_sum(z2);
      if (!(z2 > 0.0)) {
        zero = true;
      } else if (t < k) {
        xv[t] = zi / sqrt(z2);
      }
      __syncthreads();
    }
    double y2 = 0.0;
    if (!zero) {
      if (t < k) {  // ||S x|| with the final x
        double acc = 0.0;
        for (int l = t + 1; l < k; ++l) acc += mat[l * k + t] * xv[l];
        y2 = acc * acc;
      }
    }
    y2 = block_sum(y2);
    nrm = zero ? 0.0 : sqrt(y2);
  }
  if (t == 0) {
    S.orth_fro2 = fro2;
    S.orth_norm = nrm;
    if (!S.force && nrm >= a.orth_restart) S.active = 0;  // end the cycle after this step
  }
}

// ------------------------------------------------------------ tile kernels
// One workgroup per 256-row tile, one row per thread.

// Store w as basis column col: a 2-byte encoding with the scale prepared by
// the finaliser, or a plain copy for the float32 / float64 basis.
template <typename TV, typename TW>
__global__ __launch_bounds__(kBlock) void k_encode(KArgs a, int col) {
  const int s = a.tile_sys[blockIdx.x];
  if (!gated(a, s)) return;
  const float f = a.st[s].enc_f;
  const TW* w = reinterpret_cast<const TW*>(a.w);
  TV* out = reinterpret_cast<TV*>(a.V) + (int64_t)col * a.ld;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if constexpr (sizeof(TV) == 2)
    out[r] = stv<TV>(mul_rn((float)w[r], f));
  else
    out[r] = (TV)w[r];
}

// The preconditioner's arithmetic (TP) and output (TZ) types: float32 /
// float32 in the mixed modes; float64 / float64 in the float64 solver, or
// float32 / float64 when it runs with a float32 preconditioner.
template <typename TP>
__device__ __forceinline__ const TP* jacobi_dinv(const KArgs& a);
template <>
__device__ __forceinline__ const float* jacobi_dinv<float>(const KArgs& a) { return a.dinv; }
template <>
__device__ __forceinline__ const double* jacobi_dinv<double>(const KArgs& a) { return a.dinv64; }
template <typename TP>
__device__ __forceinline__ const TP* ilu_factors(const KArgs& a);
template <>
__device__ __forceinline__ const float* ilu_factors<float>(const KArgs& a) { return a.ilu32; }
template <>
__device__ __forceinline__ const double* ilu_factors<double>(const KArgs& a) { return a.ilu64; }
template <typename TP>
__device__ __forceinline__ const TP* ilu_udinv(const KArgs& a);
template <>
__device__ __forceinline__ const float* ilu_udinv<float>(const KArgs& a) { return a.iludinv; }
template <>
__device__ __forceinline__ const double* ilu_udinv<double>(const KArgs& a) { return a.iludinv64; }

// Jacobi: z_j = D^-1 v_j (or v_j once the preconditioner is switched off).
template <typename TV, typename TP, typename TZ>
__global__ __launch_bounds__(kBlock) void k_jacobi(KArgs a, int j) {
  const int s = a.tile_sys[blockIdx.x];
  if (!gated(a, s)) return;
  const TP scale = (TP)a.sc[(int64_t)s * (a.m + 1) + j];
  const bool on = a.st[s].precond_on != 0;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  // (d^-1 v) * scale: the same rounding as a sparse M = D^-1 applied by the SpMV
  const TP vr = (TP)ldv(col_ptr<TV>(a, j)[r]);
  static_cast<TZ*>(a.Z)[(int64_t)j * a.ld + r] = (TZ)(on ? (jacobi_dinv<TP>(a)[r] * vr) * scale : vr * scale);
}

// ---------------------------------------------------------- ILU(0)
// Factorisation of one dependency level (every row whose lower-triangle
// columns lie in earlier levels), one thread per row, in place on A's float64
// values: for each stored a_ik, k < i, ascending, l_ik = a_ik / u_kk, then
// every later entry a_ij of the row that row k also stores loses l_ik u_kj
// (a merge of the two sorted column lists).
__global__ __launch_bounds__(kBlock) void k_ilu_factor(KArgs a, double* __restrict__ lu,
                                                       const int32_t* __restrict__ rows, int32_t count) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= count) return;
  const int i = rows[idx];
  const int end_i = a.rp[i + 1], di = a.diagpos[i];
  for (int p = a.rp[i]; p < di; ++p) {
    const int k = a.ci[p];
    const double lik = lu[p] / lu[a.diagpos[k]];
    lu[p] = lik;
    int q = a.diagpos[k] + 1;
    const int q_end = a.rp[k + 1];
    int p2 = p + 1;
    while (q < q_end && p2 < end_i) {
      const int cq = a.ci[q], cp = a.ci[p2];
      if (cq == cp) {
        lu[p2] -= lik * lu[q];
        ++q;
        ++p2;
      } else if (cq < cp) {
        ++q;
      } else {
        ++p2;
      }
    }
  }
}

__global__ void k_ilu_finish(KArgs a, const double* __restrict__ lu, float* __restrict__ lu32,
                             float* __restrict__ dinv, double* __restrict__ dinv64) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.ld) return;
  const int b = a.rp[r], e = a.rp[r + 1];
  if (lu32)
    for (int p = b; p < e; ++p) lu32[p] = (float)lu[p];
  const double di = b < e ? 1.0 / lu[a.diagpos[r]] : 0.0;  // padding rows: zero
  if (dinv) dinv[r] = (float)di;
  if (dinv64) dinv64[r] = di;
}

// Application z_j = U^-1 L^-1 (scale_j v_j): the scaled v_j, then sweeps
// y <- v - L' y and x <- D^-1 (y - U' x) from zero starts (src = null), one
// thread per row, each row's strictly lower / upper entries in storage order.
template <typename TV, typename TP, typename TZ>
__global__ __launch_bounds__(kBlock) void k_ilu_begin(KArgs a, int j) {
  const int s = a.tile_sys[blockIdx.x];
  if (!gated(a, s)) return;
  const TP scale = (TP)a.sc[(int64_t)s * (a.m + 1) + j];
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const TP v = (TP)ldv(col_ptr<TV>(a, j)[r]) * scale;
  if (a.st[s].precond_on)
    static_cast<TP*>(a.ilu_v)[r] = v;
  else
    static_cast<TZ*>(a.Z)[(int64_t)j * a.ld + r] = (TZ)v;  // preconditioner switched off: z_j = v_j
}

template <typename TP>
__global__ __launch_bounds__(kBlock) void k_ilu_lsweep(KArgs a, const TP* __restrict__ src, TP* __restrict__ dst) {
  const int s = a.tile_sys[blockIdx.x];
  if (!gated(a, s) || (!a.st[s].precond_on && !a.st[s].force)) return;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const TP* lu = ilu_factors<TP>(a);
  TP acc = (TP)0;
  if (src)
    for (int p = a.rp[r]; p < a.diagpos[r]; ++p) acc += lu[p] * src[a.ci[p]];
  dst[r] = static_cast<const TP*>(a.ilu_v)[r] - acc;
}

template <typename TP, typename TO>
__global__ __launch_bounds__(kBlock) void k_ilu_usweep(KArgs a, const TP* __restrict__ y, const TP* __restrict__ src,
                                                       TO* __restrict__ dst) {
  const int s = a.tile_sys[blockIdx.x];
  if (!gated(a, s) || (!a.st[s].precond_on && !a.st[s].force)) return;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const TP* lu = ilu_factors<TP>(a);
  TP acc = (TP)0;
  if (src)
    for (int p = a.diagpos[r] + 1; p < a.rp[r + 1]; ++p) acc += lu[p] * src[a.ci[p]];
  dst[r] = (TO)((y[r] - acc) * ilu_udinv<TP>(a)[r]);
}

// ---------------------------------------------------- left preconditioning
// w <- M^-1 w where the system's cycle runs with the preconditioner on (or
// the state's force flag is set).  TW: w's type; TP: the preconditioner's.
__device__ __forceinline__ bool left_on(const KArgs& a, int s) {
  return gated(a, s) && (a.st[s].precond_on || a.st[s].force);
}

template <typename TW, typename TP>
__global__ __launch_bounds__(kBlock) void k_left_jacobi(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  if (!left_on(a, s)) return;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  TW* w = static_cast<TW*>(a.w);
  w[r] = (TW)(jacobi_dinv<TP>(a)[r] * (TP)w[r]);
}

template <typename TW, typename TP>
__global__ __launch_bounds__(kBlock) void k_left_ilu_begin(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  if (!left_on(a, s)) return;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  static_cast<TP*>(a.ilu_v)[r] = (TP)static_cast<const TW*>(a.w)[r];
}

template <typename TW>
__global__ __launch_bounds__(kBlock) void k_left_copy(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  if (!left_on(a, s)) return;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  static_cast<TW*>(a.w)[r] = static_cast<const TW*>(a.ptmp)[r];
}

// ||w||^2 and max|w| per tile (the preconditioned residual at a cycle's start,
// or M^-1 b): systems with a running cycle and the preconditioner on, or all
// under the force flag
template <typename TW>
__global__ __launch_bounds__(kBlock) void k_left_norm(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  const SysState& S = a.st[s];
  if (!((S.active && S.precond_on) || S.force)) return;
  const double v = (double)static_cast<const TW*>(a.w)[(int64_t)blockIdx.x * kTile + threadIdx.x];
  const double sq = block_sum(v * v);
  const double mx = block_max(fabs(v));
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = sq;
    a.part[(int64_t)a.ntile + blockIdx.x] = mx;
  }
}

template <typename TW>
__global__ __launch_bounds__(kBlock) void k_b_to_w(KArgs a) {
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  static_cast<TW*>(a.w)[r] = (TW)a.b[r];
}

// y = H^-1 s by back-substitution, one wave per system, with truncation of
// a singular leading block.  Also turns y into update coefficients.
__global__ __launch_bounds__(64) void k_backsolve(KArgs a) {
  const int s = blockIdx.x;
  SysState& S = a.st[s];
  if (!S.need_update && !S.force) return;
  const int m = a.m, M1 = m + 1;
  const int k = S.k;
  const double* Hs = a.H + (int64_t)s * M1 * m;
  const double* sv = a.s + (int64_t)s * M1;
  const int lane = threadIdx.x;
  __shared__ double ys[kMaxM];
  __shared__ int kk_s;
  double hm = 0.0;
  for (int jj = 0; jj < k; ++jj)
    for (int i = lane; i <= jj; i += 64) hm = fmax(hm, fabs(Hs[(int64_t)jj * M1 + i]));
  hm = wave_max(hm);
  if (lane == 0) {
    const double thr = 16.0 * (double)k * unit_roundoff(a.prec) * hm;
    int kk = 0;
    while (kk < k && fabs(Hs[(int64_t)kk * M1 + kk]) > thr) ++kk;
    kk_s = kk;
  }
  for (int i = lane; i < k; i += 64) ys[i] = sv[i];
  __syncthreads();
  const int kk = kk_s;
  for (int i = kk - 1; i >= 0; --i) {
    if (lane == 0) ys[i] = ys[i] / Hs[(int64_t)i * M1 + i];
    __syncthreads();
    const double yi = ys[i];
    for (int l = lane; l < i; l += 64) ys[l] -= Hs[(int64_t)i * M1 + l] * yi;
    __syncthreads();
  }
  const bool useZ = a.precond != 0 && !a.left;  // left preconditioning updates with V
  for (int i = lane; i < kk; i += 64)
    a.y[(int64_t)s * m + i] = useZ ? ys[i] : ys[i] * a.sc[(int64_t)s * M1 + i];
  if (lane == 0) {
    S.kk = kk;
    if (!S.force) S.restarts += 1;
  }
}

// x += sum_i y_i v_i (float64 accumulation over the decoded basis), or
// x += Z y in the flexible form.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_update(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  const SysState& S = a.st[s];
  if (!S.need_update && !S.force) return;
  const int kk = S.kk;
  const double* yv = a.y + (int64_t)s * a.m;
  const int64_t r = (int64_t)blockIdx.x * kTile + threadIdx.x;
  double acc = a.x[r];
  if (a.precond != 0 && !a.left && a.z64) {
    for (int i = 0; i < kk; ++i) acc += yv[i] * static_cast<const double*>(a.Z)[(int64_t)i * a.ld + r];
  } else if (a.precond != 0 && !a.left) {
    for (int i = 0; i < kk; ++i) acc += yv[i] * (double)static_cast<const float*>(a.Z)[(int64_t)i * a.ld + r];
  } else {
    for (int i = 0; i < kk; ++i) acc += yv[i] * (double)ldv(col_ptr<TV>(a, i)[r]);
  }
  a.x[r] = acc;
}

// ||b||^2 partial per tile; systems with b = 0 are done (x = 0).
__global__ __launch_bounds__(kBlock) void k_bnorm(KArgs a) {
  const double v = a.b[(int64_t)blockIdx.x * kTile + threadIdx.x];
  const double sq = block_sum(v * v);
  if (threadIdx.x == 0) a.part[blockIdx.x] = sq;
}

__global__ void k_zero_x_if_b_zero(KArgs a) {
  const int s = a.tile_sys[blockIdx.x];
  if (a.st[s].bnorm != 0.0) return;
  a.x[(int64_t)blockIdx.x * kTile + threadIdx.x] = 0.0;
}

__global__ void k_init_state(KArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  SysState S{};
  S.active = 0;
  S.status = RUNNING;
  S.best_beta = INFINITY;
  S.prev_beta = INFINITY;
  S.precond_on = a.precond != 0 ? 1 : 0;
  S.first_stall = -1;
  S.klimit = 0;
  S.orth_fro2 = 0.0;
  S.orth_norm = 0.0;
  a.st[s] = S;
}

__global__ void k_set_force(KArgs a, int on) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < a.S) a.st[s].force = on;
}

// flags a column index outside its row's own system
// bit 0 of *bad: a column outside its system; bit 1: a column more than
// 32767 away from its row (no 16-bit offset layout)
__global__ void k_check_cols(KArgs a, int32_t* bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.ld) return;
  const int s = a.tile_sys[r / kTile];
  const int64_t lo = a.sys_row0[s], hi = lo + a.sys_n[s];
  bool far = false;
  for (int k = a.rp[r]; k < a.rp[r + 1]; ++k) {
    const int64_t c = a.ci[k];
    if (c < lo || c >= hi) {
      atomicOr(bad, 1);
      return;
    }
    far = far || c - r > 32767 || r - c > 32767;
  }
  if (far) atomicOr(bad, 2);
}

__global__ void k_split_words(const double* __restrict__ src, uint32_t* __restrict__ hi,
                              uint32_t* __restrict__ lo, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = src[i];
    hi[i] = (uint32_t)__double2hiint(v);
    lo[i] = (uint32_t)__double2loint(v);
  }
}

__global__ void k_merge_words(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                              double* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = hilo_value(hi[i], lo[i]);
}

__global__ void k_convert_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) dst[k] = (float)src[k];
}

// Sum of squares of v[0, n): one partial per workgroup (grid-stride rows,
// then the fixed block tree); the host adds the partials in order.
__global__ __launch_bounds__(kBlock) void k_sumsq(const double* __restrict__ v, int64_t n, double* part) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) acc += v[k] * v[k];
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// out = float32(r * f)
__global__ void k_scale_f32(const double* __restrict__ r, int64_t n, double f, float* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) out[k] = (float)(r[k] * f);
}

__global__ void k_jacobi_setup(KArgs a, float* dinv, double* dinv64) {
  // one thread per row; padding rows (empty) get 0
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.ld) return;
  const int p0 = a.rp[r], p1 = a.rp[r + 1];
  double d = 0.0;
  for (int k = p0; k < p1; ++k)
    if (a.ci[k] == r) d += a.asplit ? hilo_value(a.ahi[k], a.alo[k]) : a.a64[k];
  const double di = (p1 > p0 && d != 0.0) ? 1.0 / d : 0.0;
  if (dinv) dinv[r] = (float)di;
  if (dinv64) dinv64[r] = di;
}

__global__ void k_shift_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int64_t n,
                            int32_t shift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) dst[k] = src[k] + shift;
}

__global__ void k_gather(const double* const* __restrict__ src, double* __restrict__ dst,
                         const int64_t* __restrict__ row0, const int32_t* __restrict__ n) {
  const int s = blockIdx.y;
  const double* p = src[s];
  const int64_t base = row0[s];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n[s];
       i += (int64_t)gridDim.x * blockDim.x)
    dst[base + i] = p[i];
}

__global__ void k_scatter(const double* __restrict__ src, double* const* __restrict__ dst,
                          const int64_t* __restrict__ row0, const int32_t* __restrict__ n) {
  const int s = blockIdx.y;
  double* p = dst[s];
  const int64_t base = row0[s];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n[s];
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = src[base + i];
}

__global__ void k_absmax(const float* __restrict__ v, int64_t n, float* part) {
  float mx = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    mx = fmaxf(mx, fabsf(v[i]));
  mx = block_max(mx);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

template <typename TV>
__global__ void k_encode_plain(const float* __restrict__ w, int64_t n, float f, TV* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = stv<TV>(mul_rn(w[i], f));
}

template <typename TV>
__global__ void k_decode_column(KArgs a, int sys, int col, double* out) {
  const int64_t row0 = a.sys_row0[sys];
  const int n = a.sys_n[sys];
  if (a.vsys) {  // normalised float32 columns, one block per system
    const float* v = static_cast<const float*>(a.V) + (int64_t)(a.m + 1) * row0 +
                     (int64_t)col * a.sys_nt[sys] * kTile;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      out[i] = (double)v[i];
    return;
  }
  const double sc = a.sc[(int64_t)sys * (a.m + 1) + col];
  const TV* v = col_ptr<TV>(a, col);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sc * (double)ldv(v[row0 + i]);
}

// ----------------------------------------------------------------- launchers

static inline int lanes_for(int ncol) {
  int L = 8;
  while (L < ncol && L < 64) L *= 2;
  return L;
}

template <typename F>
static hipError_t launch_by_prec(int prec, F&& f) {
  switch (prec) {
    case P64: return f(double{}, double{});
    case P32: return f(float{}, float{});
    case PBF16: return f(bf16_t{}, float{});
    case PF16: return f(f16_t{}, float{});
    case PL32: return f(float{}, double{});
  }
  return hipErrorInvalidValue;
}

// Resident workgroups per CU of each persistent kernel, queried once.
static std::mutex g_occ_mu;
static std::map<const void*, int> g_occ;

static int occupancy_of(const void* fn) {
  std::lock_guard<std::mutex> lock(g_occ_mu);
  auto it = g_occ.find(fn);
  if (it != g_occ.end()) return it->second;
  int nb = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  nb = std::min(nb, kMaxOcc);
  g_occ[fn] = nb;
  return nb;
}

template <typename K>
static const SegTab& split_for(const KArgs& a, K kernel) {
  return a.seg[occupancy_of(reinterpret_cast<const void*>(kernel)) - 1];
}

// Direction of the CGS passes of step j: each pass walks the basis the other
// way from the pass before it, across steps too (projection 1 of step j+1
// starts on the rows the last pass of step j touched last).
__host__ __device__ constexpr int rev_pass1(int j) { return j & 1; }
__host__ __device__ constexpr int rev_pass2(int j) { return (j & 1) ^ 1; }
__host__ __device__ constexpr int rev_pass3(int j) { return j & 1; }

// The projection kernels of a window of L columns (8, 16, 32 or 64): the
// plain ones, or with ds the variants that apply v_j's decode scale to w as
// they load it (KArgs::wsc_defer), which exist for 4- and 8-byte bases only
// (null for 2-byte ones).
template <typename TV, typename TW>
static const void* mdot_fn(int L, bool ds) {
  if (ds) {
    if constexpr (sizeof(TV) >= 4)
      return L == 8 ? (const void*)k_mdot_ds<TV, TW, 8> : L == 16 ? (const void*)k_mdot_ds<TV, TW, 16>
           : L == 32 ? (const void*)k_mdot_ds<TV, TW, 32> : (const void*)k_mdot_ds<TV, TW, 64>;
    return nullptr;
  }
  return L == 8 ? (const void*)k_mdot<TV, TW, 8> : L == 16 ? (const void*)k_mdot<TV, TW, 16>
       : L == 32 ? (const void*)k_mdot<TV, TW, 32> : (const void*)k_mdot<TV, TW, 64>;
}
// (the fused projection 2: the float64-w variant for an 8-byte w)
template <typename TV, typename TW>
static const void* axpy_mdot_fn(int L, bool ds) {
  if (ds) {
    if constexpr (sizeof(TV) < 4) {
      return nullptr;
    } else if constexpr (sizeof(TW) == 8) {
      return L == 8 ? (const void*)k_axpy_mdot64_ds<TV, TW, 8> : L == 16 ? (const void*)k_axpy_mdot64_ds<TV, TW, 16>
           : L == 32 ? (const void*)k_axpy_mdot64_ds<TV, TW, 32> : (const void*)k_axpy_mdot64_ds<TV, TW, 64>;
    } else {
      return L == 8 ? (const void*)k_axpy_mdot_ds<TV, TW, 8> : L == 16 ? (const void*)k_axpy_mdot_ds<TV, TW, 16>
           : L == 32 ? (const void*)k_axpy_mdot_ds<TV, TW, 32> : (const void*)k_axpy_mdot_ds<TV, TW, 64>;
    }
  }
  if constexpr (sizeof(TW) == 8)
    return L == 8 ? (const void*)k_axpy_mdot64<TV, TW, 8> : L == 16 ? (const void*)k_axpy_mdot64<TV, TW, 16>
         : L == 32 ? (const void*)k_axpy_mdot64<TV, TW, 32> : (const void*)k_axpy_mdot64<TV, TW, 64>;
  else
    return L == 8 ? (const void*)k_axpy_mdot<TV, TW, 8> : L == 16 ? (const void*)k_axpy_mdot<TV, TW, 16>
         : L == 32 ? (const void*)k_axpy_mdot<TV, TW, 32> : (const void*)k_axpy_mdot<TV, TW, 64>;
}

template <typename TV, typename TW, int L>
static hipError_t launch_mdot_L(const KArgs& a, int j, int col0, int mode, hipStream_t st, const SegTab** used) {
  auto go = [&](auto kern) -> hipError_t {
    const SegTab& sg = split_for(a, kern);
    hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j, col0, mode,
                       mode == 1 ? rev_pass1(j) : rev_pass2(j));
    if (used) *used = &sg;
    return hipGetLastError();
  };
  if (mode == 1 && a.wsc_defer) {
    if constexpr (sizeof(TV) >= 4) return go(k_mdot_ds<TV, TW, L>);
    else return hipErrorInvalidValue;
  }
  return go(k_mdot<TV, TW, L>);
}

template <typename TV, typename TW>
static hipError_t launch_mdot_window(const KArgs& a, int j, int col0, int mode, int L, hipStream_t st,
                                     const SegTab** used) {
  switch (L) {
    case 8: return launch_mdot_L<TV, TW, 8>(a, j, col0, mode, st, used);
    case 16: return launch_mdot_L<TV, TW, 16>(a, j, col0, mode, st, used);
    case 32: return launch_mdot_L<TV, TW, 32>(a, j, col0, mode, st, used);
    default: return launch_mdot_L<TV, TW, 64>(a, j, col0, mode, st, used);
  }
}

template <int PASS>
static hipError_t launch_fin_cols(const KArgs& a, const SegTab& sg, int j, hipStream_t st) {
  hipLaunchKernelGGL((k_fin_cols<PASS>), dim3(a.S, PASS == 1 ? j + 2 : j + 1), dim3(kBlock), 0, st, a, sg, j);
  return hipGetLastError();
}

// Arnoldi product with the values the handle chose for it: the float64
// values (or both words of the split storage) when arn64 is set, else the
// float32 copy (or the high words); LDS holds one product per non-zero of a
// row block in the kernel's accumulation type.
template <typename TX, typename TY, int MODE>
static hipError_t spmv_values(const KArgs& a, const TX* x, TY* y, int j, hipStream_t st, FinArgs fa = FinArgs{}) {
  if constexpr (MODE == SM_ARNOLDI || MODE == SM_AZ) {
    if (a.use_sell) {
      // one block per 256-row tile (4 slices), after the finaliser's blocks
      const unsigned grid = (unsigned)(a.ld / kBlock + fa.n);
      const bool d16 = a.sell_dcol != nullptr;
      if (a.arn64 && d16)
        hipLaunchKernelGGL((k_sell<double, TX, TY, MODE, true>), dim3(grid), dim3(kBlock), 0, st, a,
                           static_cast<const double*>(a.sell_val), x, y, j, fa);
      else if (a.arn64)
        hipLaunchKernelGGL((k_sell<double, TX, TY, MODE, false>), dim3(grid), dim3(kBlock), 0, st, a,
                           static_cast<const double*>(a.sell_val), x, y, j, fa);
      else if (d16)
        hipLaunchKernelGGL((k_sell<float, TX, TY, MODE, true>), dim3(grid), dim3(kBlock), 0, st, a,
                           static_cast<const float*>(a.sell_val), x, y, j, fa);
      else
        hipLaunchKernelGGL((k_sell<float, TX, TY, MODE, false>), dim3(grid), dim3(kBlock), 0, st, a,
                           static_cast<const float*>(a.sell_val), x, y, j, fa);
      return hipGetLastError();
    }
  }
  if (fa.n) return hipErrorInvalidValue;  // the finaliser rides only on the sliced product
  auto go = [&](auto kern, const auto* vals, size_t acc_bytes) {
    hipLaunchKernelGGL(kern, dim3(a.nrb), dim3(kBlock), (size_t)a.spmv_budget * acc_bytes, st, a, vals, x, y,
                       nullptr, j);
  };
  if (a.arn64) {
    if (a.asplit)
      go(k_spmv<HiLoW, TX, TY, MODE>, reinterpret_cast<const HiLoW*>(a.ahi), sizeof(AccFor<HiLoW, TY>));
    else
      go(k_spmv<double, TX, TY, MODE>, a.a64, sizeof(AccFor<double, TY>));
  } else {
    if (a.asplit)
      go(k_spmv<HiW, TX, TY, MODE>, reinterpret_cast<const HiW*>(a.ahi), sizeof(AccFor<HiW, TY>));
    else
      go(k_spmv<float, TX, TY, MODE>, a.a32, sizeof(AccFor<float, TY>));
  }
  return hipGetLastError();
}

hipError_t launch_spmv_arnoldi(const KArgs& a, int j, hipStream_t st) {
  if (a.precond != 0 && !a.left) {  // w = A z_j
    if (a.z64)
      return spmv_values<double, double, SM_AZ>(a, static_cast<const double*>(a.Z) + (int64_t)j * a.ld,
                                                (double*)a.w, j, st);
    const float* z = static_cast<const float*>(a.Z) + (int64_t)j * a.ld;
    if (wide_w(a.prec)) return spmv_values<float, double, SM_AZ>(a, z, (double*)a.w, j, st);
    return spmv_values<float, float, SM_AZ>(a, z, (float*)a.w, j, st);
  }
  return launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const TV* x = reinterpret_cast<const TV*>(a.V) + (int64_t)j * a.ld;
    return spmv_values<TV, TW, SM_ARNOLDI>(a, x, (TW*)a.w, j, st);
  });
}

hipError_t launch_ilu_factor(const KArgs& a, double* lu, const int32_t* rows, int32_t count, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_ilu_factor, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a, lu,
                       rows, count);
  return hipGetLastError();
}

hipError_t launch_ilu_finish(const KArgs& a, const double* lu, float* lu32, float* dinv, double* dinv64,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_ilu_finish, dim3((unsigned)((a.ld + 255) / 256)), dim3(256), 0, st, a, lu, lu32, dinv,
                     dinv64);
  return hipGetLastError();
}

// ILU(0) sweeps on ilu_v (L sweeps ping-pong in b0/b1, U sweeps in b2 and
// whichever of b0/b1 does not hold the L result); the last U sweep writes dst.
template <typename TP, typename TZ>
static hipError_t ilu_apply_t(const KArgs& a, TZ* dst_final, hipStream_t st) {
  TP* const b[3] = {static_cast<TP*>(a.ilu_b[0]), static_cast<TP*>(a.ilu_b[1]), static_cast<TP*>(a.ilu_b[2])};
  const TP* src = nullptr;
  for (int t = 0; t < a.ilu_sl; ++t) {
    TP* dst = b[t & 1];
    hipLaunchKernelGGL((k_ilu_lsweep<TP>), dim3(a.ntile), dim3(kBlock), 0, st, a, src, dst);
    src = dst;
  }
  const TP* y = src;
  TP* const ub[2] = {b[2], b[(a.ilu_sl & 1) ? 1 : 0]};
  const TP* usrc = nullptr;
  for (int t = 0; t < a.ilu_su; ++t) {
    if (t + 1 == a.ilu_su) {
      hipLaunchKernelGGL((k_ilu_usweep<TP, TZ>), dim3(a.ntile), dim3(kBlock), 0, st, a, y, usrc, dst_final);
    } else {
      TP* dst = ub[t & 1];
      hipLaunchKernelGGL((k_ilu_usweep<TP, TP>), dim3(a.ntile), dim3(kBlock), 0, st, a, y, usrc, dst);
      usrc = dst;
    }
  }
  return hipGetLastError();
}

// z = U^-1 L^-1 ilu_v into dst (float64 when z64, else float32)
hipError_t launch_ilu_apply(const KArgs& a, void* dst_final, hipStream_t st) {
  if (a.pc64) return ilu_apply_t<double, double>(a, static_cast<double*>(dst_final), st);
  if (a.z64) return ilu_apply_t<float, double>(a, static_cast<double*>(dst_final), st);
  return ilu_apply_t<float, float>(a, static_cast<float*>(dst_final), st);
}

// the preconditioner's (arithmetic, output) types for the handle
template <typename F>
static hipError_t launch_by_pc(const KArgs& a, F&& f) {
  if (a.pc64) return f(double{}, double{});
  if (a.z64) return f(float{}, double{});
  return f(float{}, float{});
}

hipError_t launch_precond(const KArgs& a, int j, hipStream_t st) {
  if (a.precond == 0) return hipSuccess;
  return launch_by_prec(a.prec, [&](auto tv, auto) -> hipError_t {
    using TV = decltype(tv);
    return launch_by_pc(a, [&](auto tp, auto tz) -> hipError_t {
      using TP = decltype(tp);
      using TZ = decltype(tz);
      TZ* zj = static_cast<TZ*>(a.Z) + (int64_t)j * a.ld;
      if (a.precond == 3) {
        hipLaunchKernelGGL((k_ilu_begin<TV, TP, TZ>), dim3(a.ntile), dim3(kBlock), 0, st, a, j);
        return ilu_apply_t<TP, TZ>(a, zj, st);
      }
      if (a.precond == 1) {
        hipLaunchKernelGGL((k_jacobi<TV, TP, TZ>), dim3(a.ntile), dim3(kBlock), 0, st, a, j);
      } else {
        // the learned M (float32 values) applied with the accumulation of the output's type
        const TV* x = reinterpret_cast<const TV*>(a.V) + (int64_t)j * a.ld;
        hipLaunchKernelGGL((k_spmv<float, TV, TZ, SM_PRECOND>), dim3(a.nrb), dim3(kBlock),
                           (size_t)a.spmv_budget * sizeof(AccFor<float, TZ>), st, a, a.mval, x, zj, nullptr, j);
      }
      return hipGetLastError();
    });
  });
}

// w's type for a precision mode
template <typename F>
static hipError_t launch_by_w(int prec, F&& f) {
  if (wide_w(prec)) return f(double{});
  return f(float{});
}

hipError_t launch_left_apply(const KArgs& a, hipStream_t st) {
  if (a.precond == 0 || !a.left) return hipSuccess;
  return launch_by_w(a.prec, [&](auto tw) -> hipError_t {
    using TW = decltype(tw);
    auto go = [&](auto tp) -> hipError_t {
      using TP = decltype(tp);
      if (a.precond == 1) {
        hipLaunchKernelGGL((k_left_jacobi<TW, TP>), dim3(a.ntile), dim3(kBlock), 0, st, a);
      } else if (a.precond == 3) {
        hipLaunchKernelGGL((k_left_ilu_begin<TW, TP>), dim3(a.ntile), dim3(kBlock), 0, st, a);
        return ilu_apply_t<TP, TW>(a, static_cast<TW*>(a.w), st);
      } else {
        hipLaunchKernelGGL((k_spmv<float, TW, TW, SM_LEFT>), dim3(a.nrb), dim3(kBlock),
                           (size_t)a.spmv_budget * sizeof(AccFor<float, TW>), st, a, a.mval,
                           static_cast<const TW*>(a.w), static_cast<TW*>(a.ptmp), nullptr, 0);
        hipLaunchKernelGGL((k_left_copy<TW>), dim3(a.ntile), dim3(kBlock), 0, st, a);
      }
      return hipGetLastError();
    };
    if (a.pc64) return go(double{});
    return go(float{});
  });
}

hipError_t launch_left_start(const KArgs& a, hipStream_t st) {
  if (a.precond == 0 || !a.left) return hipSuccess;
  hipError_t e = launch_left_apply(a, st);
  if (e != hipSuccess) return e;
  e = launch_by_w(a.prec, [&](auto tw) -> hipError_t {
    using TW = decltype(tw);
    hipLaunchKernelGGL((k_left_norm<TW>), dim3(a.ntile), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fin<FIN_LEFT>), dim3(a.S), dim3(kFinBlock), 0, st, a, a.part, a.ntile, a.sys_t0, a.sys_nt,
                     0);
  return hipGetLastError();
}

hipError_t launch_left_bnorm(const KArgs& a, hipStream_t st) {
  if (a.precond == 0 || !a.left) return hipSuccess;
  hipError_t e = launch_by_w(a.prec, [&](auto tw) -> hipError_t {
    using TW = decltype(tw);
    hipLaunchKernelGGL((k_b_to_w<TW>), dim3(a.ntile), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  });
  if (e == hipSuccess) e = launch_set_force(a, 1, st);
  if (e == hipSuccess) e = launch_left_apply(a, st);
  if (e == hipSuccess)
    e = launch_by_w(a.prec, [&](auto tw) -> hipError_t {
      using TW = decltype(tw);
      hipLaunchKernelGGL((k_left_norm<TW>), dim3(a.ntile), dim3(kBlock), 0, st, a);
      return hipGetLastError();
    });
  if (e == hipSuccess) e = launch_set_force(a, 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fin<FIN_BNORMP>), dim3(a.S), dim3(kFinBlock), 0, st, a, a.part, a.ntile, a.sys_t0, a.sys_nt,
                     0);
  return hipGetLastError();
}

hipError_t launch_residual(const KArgs& a, hipStream_t st, bool with_fin) {
  // z goes to w; the cycle's first basis column is written from it only
  // once the stop test has decided that a cycle starts (launch_encode)
  const size_t sh = (size_t)a.spmv_budget * 8;
  const HiLoW* hlw = reinterpret_cast<const HiLoW*>(a.ahi);
  if (wide_w(a.prec)) {
    if (a.asplit)
      hipLaunchKernelGGL((k_spmv<HiLoW, double, double, SM_RESID>), dim3(a.nrb), dim3(kBlock), sh, st, a, hlw,
                         a.x, (double*)a.w, a.b, 0);
    else
      hipLaunchKernelGGL((k_spmv<double, double, double, SM_RESID>), dim3(a.nrb), dim3(kBlock), sh, st, a,
                         a.a64, a.x, (double*)a.w, a.b, 0);
  } else {
    if (a.asplit)
      hipLaunchKernelGGL((k_spmv<HiLoW, double, float, SM_RESID>), dim3(a.nrb), dim3(kBlock), sh, st, a, hlw,
                         a.x, (float*)a.w, a.b, 0);
    else
      hipLaunchKernelGGL((k_spmv<double, double, float, SM_RESID>), dim3(a.nrb), dim3(kBlock), sh, st, a,
                         a.a64, a.x, (float*)a.w, a.b, 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !with_fin) return e;
  hipLaunchKernelGGL(k_tile_norm, dim3(a.ntile), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL((k_fin<FIN_RESID>), dim3(a.S), dim3(kFinBlock), 0, st, a, a.part, a.ntile, a.sys_t0,
                     a.sys_nt, 0);
  return hipGetLastError();
}

hipError_t launch_encode(const KArgs& a, int col, hipStream_t st) {
  return launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    hipLaunchKernelGGL((k_encode<TV, TW>), dim3(a.ntile), dim3(kBlock), 0, st, a, col);
    return hipGetLastError();
  });
}

hipError_t launch_cgs_pass1(const KArgs& a, int j, hipStream_t st, bool with_fin) {
  const SegTab* used = nullptr;
  hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const int ncol = j + 1;
    if (ncol <= 64) return launch_mdot_window<TV, TW>(a, j, 0, 1, lanes_for(ncol), st, &used);
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      hipError_t e2 = launch_mdot_window<TV, TW>(a, j, c0, 1, 64, st, &used);
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  });
  if (e != hipSuccess || !with_fin) return e;
  return launch_fin_cols<1>(a, *used, j, st);
}

template <typename TV, typename TW, int L>
static hipError_t launch_axpy_mdot_L(const KArgs& a, int j, hipStream_t st, const SegTab** used) {
  auto go = [&](auto kern) -> hipError_t {
    const SegTab& sg = split_for(a, kern);
    hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j, rev_pass2(j));
    *used = &sg;
    return hipGetLastError();
  };
  if (a.wsc_defer) {
    if constexpr (sizeof(TV) < 4) return hipErrorInvalidValue;
    else if constexpr (sizeof(TW) == 8) return go(k_axpy_mdot64_ds<TV, TW, L>);
    else return go(k_axpy_mdot_ds<TV, TW, L>);
  }
  if constexpr (sizeof(TW) == 8) return go(k_axpy_mdot64<TV, TW, L>);
  else return go(k_axpy_mdot<TV, TW, L>);
}

hipError_t launch_cgs_pass2(const KArgs& a, int j, hipStream_t st, bool with_fin) {
  const SegTab* used = nullptr;
  hipError_t e0 = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const int ncol = j + 1;
    if (ncol <= 64) {
      switch (lanes_for(ncol)) {
        case 8: return launch_axpy_mdot_L<TV, TW, 8>(a, j, st, &used);
        case 16: return launch_axpy_mdot_L<TV, TW, 16>(a, j, st, &used);
        case 32: return launch_axpy_mdot_L<TV, TW, 32>(a, j, st, &used);
        default: return launch_axpy_mdot_L<TV, TW, 64>(a, j, st, &used);
      }
    }
    if (a.wsc_defer) return hipErrorInvalidValue;  // (the split form has no deferred-scale variant)
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      auto kern = k_axpy<TV, TW, 64>;
      const SegTab& sg = split_for(a, kern);
      hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j, c0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      hipError_t e = launch_mdot_window<TV, TW>(a, j, c0, 2, 64, st, &used);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
  if (e0 != hipSuccess || !with_fin) return e0;
  return launch_fin_cols<2>(a, *used, j, st);
}

hipError_t launch_finalize_pass2(const KArgs& a, int j, hipStream_t st) {
  const SegTab* used = nullptr;
  hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    if (j + 1 <= 64) {
      const void* k = axpy_mdot_fn<TV, TW>(lanes_for(j + 1), a.wsc_defer != 0);
      if (!k) return hipErrorInvalidValue;
      used = &a.seg[occupancy_of(k) - 1];
    } else {
      used = &a.seg[occupancy_of((const void*)k_mdot<TV, TW, 64>) - 1];
    }
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  return launch_fin_cols<2>(a, *used, j, st);
}

// The split the projection-1 kernel at column j runs with (the layout of its
// partial rows, which the completing reduction reads).
static const SegTab* pass1_split(const KArgs& a, int j) {
  const SegTab* used = nullptr;
  const hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const void* k = mdot_fn<TV, TW>(j + 1 <= 64 ? lanes_for(j + 1) : 64, a.wsc_defer != 0);
    if (!k) return hipErrorInvalidValue;
    used = &a.seg[occupancy_of(k) - 1];
    return hipSuccess;
  });
  return e == hipSuccess ? used : nullptr;
}

hipError_t launch_finalize_pass1(const KArgs& a, int j, hipStream_t st) {
  const SegTab* used = pass1_split(a, j);
  if (!used) return hipErrorInvalidValue;
  return launch_fin_cols<1>(a, *used, j, st);
}

hipError_t launch_residual_finish(const KArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_tile_norm, dim3(a.ntile), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL((k_fin<FIN_RESID>), dim3(a.S), dim3(kFinBlock), 0, st, a, a.part, a.ntile, a.sys_t0,
                     a.sys_nt, 0);
  return hipGetLastError();
}

// The split of the last pass of step j (whose partial rows the per-step
// finaliser reads) and the table it wrote them to.
static const SegTab* final_split(const KArgs& a, int j, const double** src_out) {
  const SegTab* used = nullptr;
  const double* src = a.part;
  hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    if (a.ortho == 0) {
      used = &a.seg[kMgsOcc - 1];
      src = (j & 1) ? a.part : a.part2;
      return hipSuccess;
    }
    const void* k = nullptr;
    if (j + 1 <= 64) {
      const int L = lanes_for(j + 1);
      k = L == 8 ? (const void*)k_final_tile<TV, TW, 8> : L == 16 ? (const void*)k_final_tile<TV, TW, 16>
        : L == 32 ? (const void*)k_final_tile<TV, TW, 32> : (const void*)k_final_tile<TV, TW, 64>;
    } else {
      k = (const void*)k_final<TV, TW>;
    }
    used = &a.seg[occupancy_of(k) - 1];
    return hipSuccess;
  });
  if (e != hipSuccess) return nullptr;
  *src_out = src;
  return used;
}

// The per-step finaliser after the last pass of step j (k_fin_step), on the
// partial rows that pass wrote.
hipError_t launch_finalize_final(const KArgs& a, int j, hipStream_t st) {
  const double* src = nullptr;
  const SegTab* used = final_split(a, j, &src);
  if (!used) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fin_step, dim3(a.S), dim3(kBlock), 0, st, a, src, used->nseg, used->sys_sg0, used->sys_nsg, j);
  return hipGetLastError();
}

hipError_t launch_spmv_fin(const KArgs& a, int j_fin, hipStream_t st) {
  if (!a.use_sell || !a.wsc_defer || a.precond != 0 || j_fin + 1 >= a.m) return hipErrorInvalidValue;
  FinArgs fa;
  const SegTab* used = final_split(a, j_fin, &fa.src);
  if (!used) return hipErrorInvalidValue;
  fa.n = (a.S + 7) / 8 * 8;
  fa.j = j_fin;
  fa.rows = used->nseg;
  fa.r0 = used->sys_sg0;
  fa.nr = used->sys_nsg;
  const int j = j_fin + 1;
  return launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const TV* x = reinterpret_cast<const TV*>(a.V) + (int64_t)j * a.ld;
    return spmv_values<TV, TW, SM_ARNOLDI>(a, x, (TW*)a.w, j, st, fa);
  });
}

hipError_t launch_final_pass(const KArgs& a, int j, hipStream_t st, bool with_fin) {
  const SegTab* used = nullptr;
  const double* src = a.part;
  hipError_t e0 = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    if (a.ortho == 0) {  // MGS: complete dot j, then the final axpy
      auto kern = k_mgs_final<TV, TW>;
      const SegTab& sg = a.seg[kMgsOcc - 1];
      hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, sg, j);
      used = &sg;
      src = (j & 1) ? a.part : a.part2;
      return hipGetLastError();
    }
    if (j + 1 <= 64) {
      auto go = [&](auto kern) {
        const SegTab& sg = split_for(a, kern);
        hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j, rev_pass3(j));
        used = &sg;
      };
      switch (lanes_for(j + 1)) {
        case 8: go(k_final_tile<TV, TW, 8>); break;
        case 16: go(k_final_tile<TV, TW, 16>); break;
        case 32: go(k_final_tile<TV, TW, 32>); break;
        default: go(k_final_tile<TV, TW, 64>); break;
      }
    } else {
      auto kern = k_final<TV, TW>;
      const SegTab& sg = split_for(a, kern);
      hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j);
      used = &sg;
    }
    return hipGetLastError();
  });
  if (e0 != hipSuccess || !with_fin) return e0;
  hipLaunchKernelGGL(k_fin_step, dim3(a.S), dim3(kBlock), 0, st, a, src, used->nseg, used->sys_sg0, used->sys_nsg, j);
  return hipGetLastError();
}

hipError_t launch_config(const KArgs& a, int family, int j, int32_t* grid, int32_t* block, int32_t* per_cu) {
  const void* k = nullptr;
  int G = 0, B = kBlock;
  hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const int L = j + 1 <= 64 ? lanes_for(j + 1) : 64;
    switch (family) {
      case 0:  // Arnoldi SpMV: one workgroup per row block (per 256-row tile with the sliced ELL copy)
        G = a.use_sell ? (int)(a.ld / kBlock) : a.nrb;
        return hipSuccess;
      case 1:
        k = mdot_fn<TV, TW>(L, a.wsc_defer != 0);
        return k ? hipSuccess : hipErrorInvalidValue;
      case 2:
        k = j + 1 > 64 ? (const void*)k_mdot<TV, TW, 64> : axpy_mdot_fn<TV, TW>(L, a.wsc_defer != 0);
        return k ? hipSuccess : hipErrorInvalidValue;
      case 3:
        if (a.ortho == 0) {
          G = a.seg[kMgsOcc - 1].G;
          return hipSuccess;
        }
        k = j + 1 > 64 ? (const void*)k_final<TV, TW>
          : L == 8 ? (const void*)k_final_tile<TV, TW, 8> : L == 16 ? (const void*)k_final_tile<TV, TW, 16>
          : L == 32 ? (const void*)k_final_tile<TV, TW, 32> : (const void*)k_final_tile<TV, TW, 64>;
        return hipSuccess;
      case 4:
        G = a.seg[kMgsOcc - 1].G;
        return hipSuccess;
      case 5:
        G = a.nrb;
        return hipSuccess;
      case 6:
        G = a.ntile;
        return hipSuccess;
    }
    return hipErrorInvalidValue;
  });
  if (e != hipSuccess) return e;
  int occ = 0;
  if (k) {
    occ = occupancy_of(k);
    G = a.seg[occ - 1].G;
  }
  if (grid) *grid = G;
  if (block) *block = B;
  if (per_cu) *per_cu = occ;
  return hipSuccess;
}

hipError_t launch_orth_check(const KArgs& a, int j, hipStream_t st) {
  const SegTab* used = nullptr;
  hipError_t e = launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const int ncol = j + 1;
    if (ncol <= 64) return launch_mdot_window<TV, TW>(a, j, 0, 3, lanes_for(ncol), st, &used);
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      hipError_t e2 = launch_mdot_window<TV, TW>(a, j, c0, 3, 64, st, &used);
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_orth_cols, dim3(a.S, j + 1), dim3(kBlock), 0, st, a, *used, j);
  hipLaunchKernelGGL(k_orth_fin, dim3(a.S), dim3(kBlock), 0, st, a, j);
  return hipGetLastError();
}

hipError_t launch_mgs_dot(const KArgs& a, int j, int i, hipStream_t st) {
  // the next MGS launch completes this dot itself
  return launch_by_prec(a.prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    auto kern = k_mgs<TV, TW>;
    const SegTab& sg = a.seg[kMgsOcc - 1];
    hipLaunchKernelGGL(kern, dim3(sg.G), dim3(kBlock), 0, st, a, sg, j, i);
    return hipGetLastError();
  });
}

hipError_t prepare_occupancy(int prec) {
  return launch_by_prec(prec, [&](auto tv, auto tw) -> hipError_t {
    using TV = decltype(tv);
    using TW = decltype(tw);
    const void* ks[] = {
        (const void*)k_mdot<TV, TW, 8>, (const void*)k_mdot<TV, TW, 16>, (const void*)k_mdot<TV, TW, 32>,
        (const void*)k_mdot<TV, TW, 64>, (const void*)k_axpy<TV, TW, 64>,
        (const void*)k_final_tile<TV, TW, 8>, (const void*)k_final_tile<TV, TW, 16>,
        (const void*)k_final_tile<TV, TW, 32>, (const void*)k_final_tile<TV, TW, 64>,
        (const void*)k_final<TV, TW>, (const void*)k_mgs<TV, TW>, (const void*)k_mgs_final<TV, TW>};
    for (const void* k : ks) occupancy_of(k);
    // the fused projection-2 kernel in the variant that is launched, and the
    // deferred-scale variants of both projections where they exist
    for (int L : {8, 16, 32, 64}) {
      occupancy_of(axpy_mdot_fn<TV, TW>(L, false));
      if (const void* k = mdot_fn<TV, TW>(L, true)) occupancy_of(k);
      if (const void* k = axpy_mdot_fn<TV, TW>(L, true)) occupancy_of(k);
    }
    return hipSuccess;
  });
}

hipError_t launch_backsolve(const KArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_backsolve, dim3(a.S), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_update(const KArgs& a, hipStream_t st) {
  return launch_by_prec(a.prec, [&](auto tv, auto) -> hipError_t {
    using TV = decltype(tv);
    hipLaunchKernelGGL((k_update<TV>), dim3(a.ntile), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_bnorm(const KArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_bnorm, dim3(a.ntile), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL((k_fin<FIN_BNORM>), dim3(a.S), dim3(kFinBlock), 0, st, a, a.part, a.ntile, a.sys_t0,
                     a.sys_nt, 0);
  hipLaunchKernelGGL(k_zero_x_if_b_zero, dim3(a.ntile), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_init_state(const KArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_init_state, dim3((a.S + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_set_force(const KArgs& a, int on, hipStream_t st) {
  hipLaunchKernelGGL(k_set_force, dim3((a.S + 255) / 256), dim3(256), 0, st, a, on);
  return hipGetLastError();
}

hipError_t launch_check_cols(const KArgs& a, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_check_cols, dim3((unsigned)((a.ld + 255) / 256)), dim3(256), 0, st, a, bad);
  return hipGetLastError();
}

hipError_t launch_split_words(const double* src, uint32_t* hi, uint32_t* lo, int64_t n, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (blocks > 0) hipLaunchKernelGGL(k_split_words, dim3((unsigned)blocks), dim3(256), 0, st, src, hi, lo, n);
  return hipGetLastError();
}

hipError_t launch_merge_words(const uint32_t* hi, const uint32_t* lo, double* dst, int64_t n, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (blocks > 0) hipLaunchKernelGGL(k_merge_words, dim3((unsigned)blocks), dim3(256), 0, st, hi, lo, dst, n);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (blocks > 0) hipLaunchKernelGGL(k_convert_f32, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* v, int64_t n, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(nblk), dim3(kBlock), 0, st, v, n, part);
  return hipGetLastError();
}

hipError_t launch_scale_f32(const double* r, int64_t n, double f, float* out, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  if (blocks > 0) hipLaunchKernelGGL(k_scale_f32, dim3(blocks), dim3(256), 0, st, r, n, f, out);
  return hipGetLastError();
}

hipError_t launch_jacobi_setup(const KArgs& a, float* dinv, double* dinv64, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_setup, dim3((unsigned)((a.ld + 255) / 256)), dim3(256), 0, st, a, dinv, dinv64);
  return hipGetLastError();
}

hipError_t launch_spmv_plain(const KArgs& a, int prec, const void* x, void* y, hipStream_t st) {
  const size_t sh8 = (size_t)a.spmv_budget * 8, sh4 = (size_t)a.spmv_budget * 4;
  if (prec == P64) {
    if (a.asplit)
      hipLaunchKernelGGL((k_spmv<HiLoW, double, double, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh8, st, a,
                         reinterpret_cast<const HiLoW*>(a.ahi), (const double*)x, (double*)y, nullptr, 0);
    else
      hipLaunchKernelGGL((k_spmv<double, double, double, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh8, st, a,
                         a.a64, (const double*)x, (double*)y, nullptr, 0);
  } else if (prec == PL32) {  // float32 values and x, float64 sums and y
    if (a.asplit)
      hipLaunchKernelGGL((k_spmv<HiW, float, double, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh8, st, a,
                         reinterpret_cast<const HiW*>(a.ahi), (const float*)x, (double*)y, nullptr, 0);
    else
      hipLaunchKernelGGL((k_spmv<float, float, double, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh8, st, a,
                         a.a32, (const float*)x, (double*)y, nullptr, 0);
  } else {
    if (a.asplit)
      hipLaunchKernelGGL((k_spmv<HiW, float, float, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh4, st, a,
                         reinterpret_cast<const HiW*>(a.ahi), (const float*)x, (float*)y, nullptr, 0);
    else
      hipLaunchKernelGGL((k_spmv<float, float, float, SM_PLAIN>), dim3(a.nrb), dim3(kBlock), sh4, st, a,
                         a.a32, (const float*)x, (float*)y, nullptr, 0);
  }
  return hipGetLastError();
}

hipError_t launch_build_sell(const KArgs& a, const void* vals, int v32, void* sv, int32_t* sc, int16_t* sd,
                             uint8_t* sl, hipStream_t st) {
  hipLaunchKernelGGL(k_build_sell, dim3((unsigned)((a.ld + 255) / 256)), dim3(256), 0, st, a, vals, v32, sv, sc,
                     sd, sl);
  return hipGetLastError();
}

hipError_t launch_residual_plain(const KArgs& a, const double* b, const double* x, double* r,
                                 hipStream_t st) {
  const size_t sh = (size_t)a.spmv_budget * 8;
  if (a.asplit)
    hipLaunchKernelGGL((k_spmv<HiLoW, double, double, SM_RESID_PLAIN>), dim3(a.nrb), dim3(kBlock), sh, st, a,
                       reinterpret_cast<const HiLoW*>(a.ahi), x, r, b, 0);
  else
    hipLaunchKernelGGL((k_spmv<double, double, double, SM_RESID_PLAIN>), dim3(a.nrb), dim3(kBlock), sh, st, a,
                       a.a64, x, r, b, 0);
  return hipGetLastError();
}

hipError_t launch_absmax(const float* w, int64_t n, float* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_absmax, dim3(nblk), dim3(kBlock), 0, st, w, n, part);
  return hipGetLastError();
}

hipError_t launch_encode_plain(int prec, int64_t n, const float* w, float f, void* out, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  if (blocks == 0) return hipSuccess;
  if (prec == PBF16)
    hipLaunchKernelGGL((k_encode_plain<bf16_t>), dim3(blocks), dim3(256), 0, st, w, n, f, (bf16_t*)out);
  else
    hipLaunchKernelGGL((k_encode_plain<f16_t>), dim3(blocks), dim3(256), 0, st, w, n, f, (f16_t*)out);
  return hipGetLastError();
}

hipError_t launch_decode_column(const KArgs& a, int sys, int col, double* out, hipStream_t st) {
  return launch_by_prec(a.prec, [&](auto tv, auto) -> hipError_t {
    using TV = decltype(tv);
    hipLaunchKernelGGL((k_decode_column<TV>), dim3(256), dim3(256), 0, st, a, sys, col, out);
    return hipGetLastError();
  });
}

hipError_t launch_shift_cols(const int32_t* src, int32_t* dst, int64_t nnz, int32_t shift, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<int64_t>((nnz + 255) / 256, 65536);
  if (blocks > 0) hipLaunchKernelGGL(k_shift_i32, dim3(blocks), dim3(256), 0, st, src, dst, nnz, shift);
  return hipGetLastError();
}

hipError_t launch_gather(const double* const* src, double* dst, const int64_t* row0, const int32_t* n,
                         int S, int64_t maxn, hipStream_t st) {
  const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((maxn + 255) / 256, 1024));
  hipLaunchKernelGGL(k_gather, dim3(bx, S), dim3(256), 0, st, src, dst, row0, n);
  return hipGetLastError();
}

hipError_t launch_scatter(const double* src, double* const* dst, const int64_t* row0, const int32_t* n,
                          int S, int64_t maxn, hipStream_t st) {
  const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((maxn + 255) / 256, 1024));
  hipLaunchKernelGGL(k_scatter, dim3(bx, S), dim3(256), 0, st, src, dst, row0, n);
  return hipGetLastError();
}

}  // namespace gm

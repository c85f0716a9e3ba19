// Persistent batch schedule of restarted GMRES(m) for gfx950: one workgroup
// of 1024 threads solves one system from start to finish, and workgroups
// take systems from a queue (largest first) until it is empty, all in one
// kernel launch.
//
// Per system (Algorithm 1 with MGS, float32 Arnoldi, float64 residual,
// update, Hessenberg matrix and rotations): the work vector w lives in
// registers, R = ceil(n / 1024) rows per thread (n <= 65,536), and each
// basis vector is kept in LDS between its dot product and its axpy (up to
// 34 rows per thread), so an MGS step reads v_i once from memory (for n up
// to 34,816; larger systems re-read the rest) and never streams w; H, the rotations
// and the least-squares right-hand side live in LDS; the basis lives in
// HBM in one contiguous block per system.  Every reduction is a fixed-order
// block sum (per-thread float32 partials, float64 across threads), so a
// system's result does not depend on the other systems of the batch or on
// which workgroup ran it.
#include <math.h>

#include <algorithm>

#include "gmres_internal.hpp"

namespace gm {
namespace {

constexpr int kPB = 1024;        // threads per system
constexpr int kPW = kPB / 64;    // waves per system
constexpr int kStage = 34;       // rows per thread of v_i kept in LDS between an MGS dot and its axpy
constexpr int kStageLd = kStage + 1;  // odd row stride: lanes hit distinct banks, one base address

struct PShared {
  double red[2][kPW][2];               // double-buffered wave partials (two sums each)
  double H[kMaxPM * (kMaxPM + 1) / 2];  // rotated Hessenberg matrix, packed upper triangle by columns
  double cs[kMaxPM], sn[kMaxPM], sv[kMaxPM + 1], y[kMaxPM], ar[kMaxPM + 1];
  int ctl[4];
  double dctl[2];
  int sys;
  float vst[kPB][kStageLd];            // staged rows of v_i (thread t owns row t)
};

// column j of the rotated H (rows 0..j) starts at j (j + 1) / 2
__device__ __forceinline__ int hoff(int j) { return j * (j + 1) / 2; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over the workgroup of (u, v), identical in every thread; `buf`
// alternates between calls so one barrier per call suffices.
__device__ __forceinline__ void bsum2(PShared& sh, int& buf, double& u, double& v) {
  u = wsum(u);
  v = wsum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh.red[buf][w][0] = u;
    sh.red[buf][w][1] = v;
  }
  __syncthreads();
  double su = 0.0, sv = 0.0;
#pragma unroll
  for (int q = 0; q < kPW; ++q) {
    su += sh.red[buf][q][0];
    sv += sh.red[buf][q][1];
  }
  u = su;
  v = sv;
  buf ^= 1;
}

__device__ __forceinline__ double bsum(PShared& sh, int& buf, double u) {
  double v = 0.0;
  bsum2(sh, buf, u, v);
  return u;
}

__device__ __forceinline__ void p_givens(double a, double b, double& c, double& s) {
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double rho = hypot(a, b);
  c = a / rho;
  s = b / rho;
}

// Buffer resources: every thread addresses its rows as one 32-bit lane
// offset plus a scalar offset per row group, so R rows per thread cost no
// per-row 64-bit addresses (the kernel runs at 128 registers per thread).
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t mkr(const void* base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           (int)(uint32_t)std::min<uint64_t>(bytes, 0xffffffffu), 0x00020000);
}
__device__ __forceinline__ float ldf(rsrc_t r, uint32_t vo, uint32_t so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ int ldi(rsrc_t r, uint32_t vo, uint32_t so) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ double ldd(rsrc_t r, uint32_t vo, uint32_t so) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
// The same load with the non-temporal hint, for a value read once.  Being a
// different load, it is never merged with a later ordinary load of the same
// address (the right-hand side read for ||b||, merged with every restart
// residual's read of it, would keep R float64 values live for the solve).
__device__ __forceinline__ double ldd_once(rsrc_t r, uint32_t vo, uint32_t so) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 2);
  return __hiloint2double((int)v[1], (int)v[0]);
}
__device__ __forceinline__ int ldu8(rsrc_t r, uint32_t vo, uint32_t so) {
  return (int)__builtin_amdgcn_raw_buffer_load_b8(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ int ldu16(rsrc_t r, uint32_t vo, uint32_t so) {
  return (int)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void stf(float x, rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void std64(double x, rsrc_t r, uint32_t vo, uint32_t so) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)vo, (int)so, 0);
}

// Values that are the same in every lane, pinned to scalar registers: buffer
// descriptors built from them must be scalar, else every access becomes a
// loop over lanes.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// What the persistent kernel reads, packed: the fields it uses of the
// engine's argument block, in one small kernel-argument block (the full
// block keeps more scalar registers live and spills them).
struct PArgs {
  const int32_t* rp;
  const int32_t* ci;
  const float* a32;
  const double* a64;
  float* V;
  double* x;
  const double* b;
  double* Hbar;
  double* hist;
  SysState* st;
  const int64_t* sys_row0;
  const int32_t* sys_n;
  const int32_t* sys_nt;
  const float* ell_val;
  const uint16_t* ell_col;
  const uint8_t* ell_len;
  const int64_t* ell_off;
  const int32_t* ell_w;
  double tol;
  double restart_improve;
  int64_t max_iters;
  int64_t ld;
  int32_t S;
  int32_t m;
  int32_t stall_cycles;
  int32_t stall_win;
  int32_t restart_repeat;
  int32_t restart_on_stall;
};

PArgs pargs_of(const KArgs& k) {
  PArgs p;
  p.rp = k.rp;
  p.ci = k.ci;
  p.a32 = k.a32;
  p.a64 = k.a64;
  p.V = static_cast<float*>(k.V);
  p.x = k.x;
  p.b = k.b;
  p.Hbar = k.Hbar;
  p.hist = k.hist;
  p.st = k.st;
  p.sys_row0 = k.sys_row0;
  p.sys_n = k.sys_n;
  p.sys_nt = k.sys_nt;
  p.ell_val = k.ell_val;
  p.ell_col = k.ell_col;
  p.ell_len = k.ell_len;
  p.ell_off = k.ell_off;
  p.ell_w = k.ell_w;
  p.tol = k.tol;
  p.restart_improve = k.restart_improve;
  p.max_iters = k.max_iters;
  p.ld = k.ld;
  p.S = k.S;
  p.m = k.m;
  p.stall_cycles = k.stall_cycles;
  p.stall_win = k.stall_win;
  p.restart_repeat = k.restart_repeat;
  p.restart_on_stall = k.restart_on_stall;
  return p;
}

// The descriptors of one system's Arnoldi SpMV (the ones its variant reads).
struct SpmvSys {
  rsrc_t r0, r1, r2;  // CSR: row pointers of the system, columns, values; ELL: values, columns, lengths
  int col0;           // global column of the system's first row
  int ew;             // ELL width
  uint32_t pn;        // padded rows (ELL slice stride)
};

// rpr, cir: the system's row-pointer and column descriptors, which the
// float64 residual reads too (the CSR variants share them).
template <int PV>
__device__ __forceinline__ SpmvSys spmv_sys_of(const PArgs& a, int s, int64_t row0, int n, uint32_t pn,
                                              uint32_t nz_end, rsrc_t rpr, rsrc_t cir) {
  SpmvSys m;
  m.col0 = (int)row0;
  m.pn = pn;
  m.ew = 0;
  if constexpr (PV == PV_ELL16) {
    const int64_t off = uni64(a.ell_off[s]);
    m.ew = uni(a.ell_w[s]);
    m.r0 = mkr(a.ell_val + off, (uint64_t)m.ew * pn * 4);
    m.r1 = mkr(a.ell_col + off, (uint64_t)m.ew * pn * 2);
    m.r2 = mkr(a.ell_len + row0, (uint64_t)n);
  } else {
    m.r0 = rpr;
    m.r1 = cir;
    m.r2 = mkr(a.a32, (uint64_t)nz_end * 4);
  }
  return m;
}

// A batch of B loads of a basis column (rows q0 .. q0 + B - 1 of this
// thread) issued together.  At the register ceiling the scheduler would
// otherwise interleave each load with its use (one round trip per row); the
// empty asm takes every loaded value as an input, so all B are complete
// before the first is used and they go out back to back.
template <int B>
__device__ __forceinline__ void load_rows(float (&v)[B], rsrc_t r, uint32_t t4, int q0) {
#pragma unroll
  for (int e = 0; e < B; ++e) v[e] = ldf(r, t4, (uint32_t)(q0 + e) * kPB * 4u);
  if constexpr (B == 16)
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]),
                 "v"(v[8]), "v"(v[9]), "v"(v[10]), "v"(v[11]), "v"(v[12]), "v"(v[13]), "v"(v[14]), "v"(v[15]));
  else if constexpr (B == 8)
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
  else if constexpr (B == 4)
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]));
  else if constexpr (B == 2)
    asm volatile("" ::"v"(v[0]), "v"(v[1]));
  else
    asm volatile("" ::"v"(v[0]));
}

// w = A x over the system's rows (row q of thread t is t + 1024 q), entries in
// groups of G, each row's products added in storage order; entries past a
// row are masked (their gathers may fall anywhere, or past x).
template <int R, int G>
__device__ __forceinline__ void spmv_csr(const SpmvSys& m, rsrc_t x, float (&w)[R]) {
  const uint32_t t4 = threadIdx.x * 4u;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const uint32_t so = (uint32_t)q * kPB * 4u;
    const int k0 = ldi(m.r0, t4, so), k1 = ldi(m.r0, t4, so + 4u);
    float acc = 0.f;
    for (int kb = k0; kb < k1; kb += G) {
      float av[G];
      int cv[G];
#pragma unroll
      for (int e = 0; e < G; ++e) {
        av[e] = ldf(m.r2, (uint32_t)(kb + e) * 4u, 0);
        cv[e] = ldi(m.r1, (uint32_t)(kb + e) * 4u, 0);
      }
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const float xv = ldf(x, (uint32_t)(cv[e] - m.col0) * 4u, 0);
        if (kb + e < k1) acc += av[e] * xv;
      }
    }
    w[q] = acc;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The same products from the ELL copy: slice k holds entry k of every row,
// so each load of the workgroup is contiguous; slices are read in groups of
// 8 (a group reaching past the last slice reads zeros through the bounded
// descriptor, and the row length masks them).
template <int R>
__device__ __forceinline__ void spmv_ell(const SpmvSys& m, rsrc_t x, float (&w)[R]) {
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const uint32_t r = (uint32_t)q * kPB;
    const int len = ldu8(m.r2, t, r);  // rows past n: zero
    float acc = 0.f;
    for (int kb = 0; kb < m.ew; kb += 8) {
      float av[8];
      int cv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t so = (uint32_t)(kb + e) * m.pn + r;
        av[e] = ldf(m.r0, t * 4u, so * 4u);
        cv[e] = ldu16(m.r1, t * 2u, so * 2u);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float xv = ldf(x, (uint32_t)cv[e] * 4u, 0);
        if (kb + e < len) acc += av[e] * xv;
      }
    }
    w[q] = acc;
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int R, int PV>
__device__ __forceinline__ void spmv_sys(const SpmvSys& m, rsrc_t x, float (&w)[R]) {
  if constexpr (PV == PV_ELL16)
    spmv_ell<R>(m, x, w);
  else if constexpr (PV == PV_CSR4)
    spmv_csr<R, 4>(m, x, w);
  else
    spmv_csr<R, 8>(m, x, w);
}

// Row q of thread t is r = t + 1024 q.  Every vector of the system is read
// and written through a descriptor bounded to its n rows: loads past the end
// return zero and stores past it are dropped, so the row loops need no
// guards and a thread keeps up to 16 loads in flight.
template <int R, int PV>
__device__ __forceinline__ void p_system(const PArgs& a, int s, PShared& sh) {
  const int t = threadIdx.x;
  const int m = a.m, M1 = m + 1;
  const int64_t row0 = uni64(a.sys_row0[s]);
  const int n = uni(a.sys_n[s]);
  const uint32_t pn = (uint32_t)uni(a.sys_nt[s]) * kTile;  // column stride of this system's basis
  const uint32_t nz_end = (uint32_t)uni(a.rp[row0 + n]);    // entries of systems up to this one
  float* Vs = a.V + (int64_t)M1 * row0;
  auto col = [&](int i) { return mkr(Vs + (size_t)i * pn, (uint64_t)n * 4); };
  const rsrc_t rpr = mkr(a.rp + row0, (uint64_t)(n + 1) * 4);
  const rsrc_t cir = mkr(a.ci, (uint64_t)nz_end * 4);
  const rsrc_t a64r = mkr(a.a64, (uint64_t)nz_end * 8);
  const SpmvSys sm = spmv_sys_of<PV>(a, s, row0, n, pn, nz_end, rpr, cir);
  const rsrc_t xall = mkr(a.x, (uint64_t)a.ld * 8);         // gathers by global column
  const rsrc_t xs = mkr(a.x + row0, (uint64_t)n * 8);       // this system's rows
  const rsrc_t br = mkr(a.b + row0, (uint64_t)n * 8);
  double* hbar = a.Hbar + (int64_t)s * M1 * m;
  const uint32_t t4 = (uint32_t)t * 4u, t8 = (uint32_t)t * 8u;
  const int col0 = (int)row0;  // global column of local row 0
  int buf = 0;
  float w[R];

  double bb = 0.0, dummy = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double bv = ldd_once(br, t8, (uint32_t)q * kPB * 8u);
    bb += bv * bv;
  }
  bsum2(sh, buf, bb, dummy);
  const double bnorm = sqrt(bb);

  int status = RUNNING, nhist = 0, cycle = 0, no_progress = 0, first_stall = -1, klast = 0, klimit = 0;
  int64_t iters = 0, restarts = 0;
  double best = INFINITY, beta = 0.0, rel = 0.0;
  if (bnorm == 0.0) {
#pragma unroll
    for (int q = 0; q < R; ++q) std64(0.0, xs, t8, (uint32_t)q * kPB * 8u);
    status = CONVERGED;
  }
  const double bd_u = 0x1p-24;
  while (status == RUNNING) {
    // ---- float64 restart residual z = b - A x, beta, stop tests, v_1
    double zz = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t so = (uint32_t)q * kPB * 4u;
      const int k0 = ldi(rpr, t4, so), k1 = ldi(rpr, t4, so + 4u);  // rows past n: empty
      double acc = 0.0;
      for (int kb = k0; kb < k1; kb += 4) {
        double av[4];
        int cv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          av[e] = ldd(a64r, (uint32_t)(kb + e) * 8u, 0);
          cv[e] = ldi(cir, (uint32_t)(kb + e) * 4u, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double xv = ldd(xall, (uint32_t)cv[e] * 8u, 0);
          if (kb + e < k1) acc += av[e] * xv;
        }
      }
      const double z = ldd(br, t8, (uint32_t)q * kPB * 8u) - acc;  // zero past n
      zz += z * z;
      w[q] = (float)z;
      // one row at a time, bounded registers: the empty asm consumes zz here,
      // so the subtraction is not sunk past the other rows' loops (which
      // would keep every row's float64 sum live at once)
      asm volatile("" : "+v"(zz));
      __builtin_amdgcn_sched_barrier(0);
    }
    bsum2(sh, buf, zz, dummy);
    beta = sqrt(zz);
    rel = beta / bnorm;
    if (t == 0 && nhist < kHistCap) a.hist[(int64_t)s * kHistCap + nhist] = rel;
    ++nhist;
    if (rel <= a.tol) {
      status = CONVERGED;
      break;
    }
    if (!isfinite(beta)) {
      status = STALLED;
      break;
    }
    if (iters >= a.max_iters) {
      status = MAXITER;
      break;
    }
    no_progress = beta >= best ? no_progress + 1 : 0;
    best = fmin(best, beta);
    if (no_progress >= a.stall_cycles) {
      status = STALLED;
      break;
    }
    ++cycle;
    {
      const float inv = (float)(1.0 / beta);
      const rsrc_t v0 = col(0);
#pragma unroll
      for (int q = 0; q < R; ++q) stf(w[q] * inv, v0, t4, (uint32_t)q * kPB * 4u);
    }
    if (t == 0) {
      sh.sv[0] = beta;
      sh.ar[0] = beta;
    }
    int k = 0;
    for (int j = 0; j < m; ++j) {
      __syncthreads();  // v_j complete (stores of every thread)
      const rsrc_t vj = col(j);
      // ---- w = A v_j (float32), in the system's tuned SpMV variant
      spmv_sys<R, PV>(sm, vj, w);
      float wp = 0.f;
#pragma unroll
      for (int q = 0; q < R; ++q) wp += w[q] * w[q];
      double wsq = (double)wp;
      // ---- modified Gram-Schmidt: h_ij = w . v_i, w -= h_ij v_i
      double wnorm_pre = 0.0;
      for (int i = 0; i <= j; ++i) {
        const rsrc_t vi = col(i);
        // w . v_i in batches of 16 rows: the batch's loads go out together,
        // its products are summed in row order, then the rows kept for the
        // update are staged in LDS (read back by this thread only: no
        // barrier).  The staging stores come after the batch's products: with
        // them interleaved the compiler reused store data registers a few
        // instructions after each store, and the 64-row tier computed wrong
        // sums (not seen in this order).
        float d = 0.f;
        constexpr int B = R < 16 ? R : 16;
#pragma unroll
        for (int q0 = 0; q0 < R; q0 += B) {
          float vb[B];
          load_rows<B>(vb, vi, t4, q0);
#pragma unroll
          for (int e = 0; e < B; ++e) d += w[q0 + e] * vb[e];
#pragma unroll
          for (int e = 0; e < B; ++e)
            if (q0 + e < kStage) sh.vst[t][q0 + e] = vb[e];
          __builtin_amdgcn_sched_barrier(0);
        }
        double h = (double)d;
        if (i == 0) {
          bsum2(sh, buf, h, wsq);
          wnorm_pre = sqrt(wsq);
        } else {
          h = bsum(sh, buf, h);
        }
        if (t == 0) {
          sh.H[hoff(j) + i] = h;
          hbar[(int64_t)j * M1 + i] = h;
        }
        const float hf = (float)h;
        // rows staged in LDS, then the rest reloaded in batches of 16 (the
        // last batch ends at row R - 1 and skips rows already updated)
#pragma unroll
        for (int q = 0; q < (R < kStage ? R : kStage); ++q) w[q] -= hf * sh.vst[t][q];
        if constexpr (R > kStage) {
#pragma unroll
          for (int q0 = kStage; q0 < R; q0 += 16) {
            const int base = q0 < R - 16 ? q0 : R - 16;
            float vb[16];
            load_rows<16>(vb, vi, t4, base);
#pragma unroll
            for (int e = 0; e < 16; ++e)
              if (base + e >= q0) w[base + e] -= hf * vb[e];
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      float ws = 0.f;
#pragma unroll
      for (int q = 0; q < R; ++q) ws += w[q] * w[q];
      const double hn = sqrt(bsum(sh, buf, (double)ws));
      ++iters;
      k = j + 1;
      // ---- Givens rotations of column j, stop decisions (one lane)
      if (t == 0) {
        hbar[(int64_t)j * M1 + j + 1] = hn;
        double* hc = sh.H + hoff(j);
        double cur = hc[0];
        for (int i = 0; i < j; ++i) {
          const double nxt = hc[i + 1];
          hc[i] = sh.cs[i] * cur + sh.sn[i] * nxt;
          cur = -sh.sn[i] * cur + sh.cs[i] * nxt;
        }
        double c, sg;
        p_givens(cur, hn, c, sg);
        sh.cs[j] = c;
        sh.sn[j] = sg;
        const double sjv = sh.sv[j];
        sh.sv[j + 1] = -sg * sjv;
        sh.sv[j] = c * sjv;
        hc[j] = c * cur + sg * hn;
        const double res = fabs(sg * sjv);
        sh.ar[j + 1] = res;
        if (cycle == 1 && first_stall < 0) {
          const int J = j + 1 - a.stall_win;
          if (J >= 0 && res > sh.ar[J] / 1.001) first_stall = J;
        }
        const double bd = 16.0 * (double)(j + 1) * bd_u;
        const bool fin = isfinite(hn) && isfinite(cur);
        const bool first_stage = !a.restart_repeat || klimit == 0;
        const int Js = j + 1 - a.stall_win;
        const bool end = !fin || (j + 1 >= m) || !(hn > bd * wnorm_pre) || res <= a.tol * bnorm ||
                         iters >= a.max_iters ||
                         (a.restart_improve > 0.0 && first_stage && res <= a.restart_improve * beta) ||
                         (!first_stage && j + 1 >= klimit) ||
                         (a.restart_on_stall && Js >= 0 && res > sh.ar[Js] / 1.001);
        if (end && a.restart_repeat && klimit == 0) klimit = fin ? j + 1 : j;
        sh.ctl[0] = end ? 1 : 0;
        sh.ctl[1] = fin ? 1 : 0;
      }
      __syncthreads();
      const bool end = sh.ctl[0] != 0;
      if (sh.ctl[1] == 0) {  // non-finite column: the cycle keeps the columns before it
        k = j;
        break;
      }
      if (hn > 0.0) {
        const float inv = (float)(1.0 / hn);
        const rsrc_t vn = col(j + 1);
#pragma unroll
        for (int q = 0; q < R; ++q) stf(w[q] * inv, vn, t4, (uint32_t)q * kPB * 4u);
      }
      if (end) break;
    }
    klast = k;
    if (k == 0) continue;  // nothing to apply: the next residual decides (stall after stall_cycles)
    // ---- back-substitution y = H_k^-1 s_k with truncation of a singular leading block (one lane)
    if (t == 0) {
      double hm = 0.0;
      for (int jj = 0; jj < k; ++jj)
        for (int i = 0; i <= jj; ++i) hm = fmax(hm, fabs(sh.H[hoff(jj) + i]));
      const double thr = 16.0 * (double)k * bd_u * hm;
      int kk = 0;
      while (kk < k && fabs(sh.H[hoff(kk) + kk]) > thr) ++kk;
      for (int i = 0; i < kk; ++i) sh.y[i] = sh.sv[i];
      for (int i = kk - 1; i >= 0; --i) {
        sh.y[i] /= sh.H[hoff(i) + i];
        for (int l = 0; l < i; ++l) sh.y[l] -= sh.H[hoff(i) + l] * sh.y[i];
      }
      sh.ctl[2] = kk;
    }
    __syncthreads();
    const int kk = sh.ctl[2];
    // ---- x += sum_i y_i v_i (float64 accumulation)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint32_t xo = (uint32_t)q * kPB * 8u;
      double acc = ldd(xs, t8, xo);
      for (int i = 0; i < kk; ++i) acc += sh.y[i] * (double)ldf(col(i), t4, (uint32_t)q * kPB * 4u);
      std64(acc, xs, t8, xo);
      __builtin_amdgcn_sched_barrier(0);
    }
    ++restarts;
    __syncthreads();  // x complete before the next residual reads it
  }
  if (t == 0) {
    SysState& S = a.st[s];
    S.status = status;
    S.iters = iters;
    S.restarts = restarts;
    S.bnorm = bnorm;
    S.beta = beta;
    S.rel = bnorm == 0.0 ? 0.0 : rel;
    S.first_stall = first_stall;
    S.nhist = nhist;
    S.k = klast;
    S.cycle = cycle;
    S.active = 0;
  }
  __syncthreads();  // the next system reuses the shared state
}

template <int PV>
__global__ __launch_bounds__(kPB) void k_batch_persistent(PArgs a, const int32_t* __restrict__ order,
                                                          int32_t* counter) {
  __shared__ PShared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.sys = atomicAdd(counter, 1);
    __syncthreads();
    // the whole workgroup works on one system: keep its index in scalar
    // registers (read through LDS it would look divergent, and every buffer
    // descriptor built from it would need a per-lane loop)
    const int q = __builtin_amdgcn_readfirstlane(sh.sys);
    __syncthreads();
    if (q >= a.S) break;
    const int s = __builtin_amdgcn_readfirstlane(order[q]);
    const int rows = (a.sys_n[s] + kPB - 1) / kPB;
    if (rows <= 1) p_system<1, PV>(a, s, sh);
    else if (rows <= 2) p_system<2, PV>(a, s, sh);
    else if (rows <= 4) p_system<4, PV>(a, s, sh);
    else if (rows <= 8) p_system<8, PV>(a, s, sh);
    else if (rows <= 16) p_system<16, PV>(a, s, sh);
    else if (rows <= 32) p_system<32, PV>(a, s, sh);
    else p_system<kMaxPR, PV>(a, s, sh);
  }
}

__global__ void k_build_ell(KArgs a, int64_t row0, int n, int w, int pn, float* __restrict__ val,
                            uint16_t* __restrict__ col, uint8_t* __restrict__ len) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= pn) return;
  const int p0 = r < n ? a.rp[row0 + r] : 0, p1 = r < n ? a.rp[row0 + r + 1] : 0;
  for (int k = 0; k < w; ++k) {
    const int p = p0 + k;
    val[(int64_t)k * pn + r] = p < p1 ? a.a32[p] : 0.0f;
    col[(int64_t)k * pn + r] = p < p1 ? (uint16_t)(a.ci[p] - row0) : (uint16_t)0;
  }
  if (r < n) len[row0 + r] = (uint8_t)(p1 - p0);
}

__global__ void k_counter_clear(int32_t* counter) { counter[0] = 0; }

}  // namespace

hipError_t launch_build_ell(const KArgs& a, int s, int64_t row0, int n, int w, int64_t off, int pn,
                            float* val, uint16_t* col, uint8_t* len, hipStream_t st) {
  (void)s;
  hipLaunchKernelGGL(k_build_ell, dim3((pn + 255) / 256), dim3(256), 0, st, a, row0, n, w, pn, val + off,
                     col + off, len);
  return hipGetLastError();
}

hipError_t launch_batch_persistent(const KArgs& a, const int32_t* order, int32_t* counter, int pv, hipStream_t st) {
  const int grid = std::max(1, std::min(a.S, a.ncu));
  const PArgs p = pargs_of(a);
  hipLaunchKernelGGL(k_counter_clear, dim3(1), dim3(1), 0, st, counter);
  switch (pv) {
    case PV_CSR4:
      hipLaunchKernelGGL(k_batch_persistent<PV_CSR4>, dim3(grid), dim3(kPB), 0, st, p, order, counter);
      break;
    case PV_ELL16:
      hipLaunchKernelGGL(k_batch_persistent<PV_ELL16>, dim3(grid), dim3(kPB), 0, st, p, order, counter);
      break;
    default:
      hipLaunchKernelGGL(k_batch_persistent<PV_CSR8>, dim3(grid), dim3(kPB), 0, st, p, order, counter);
  }
  return hipGetLastError();
}

}  // namespace gm

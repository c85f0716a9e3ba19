// Kernels of the learned sparse approximate inverse for gfx950 (wave64).
//
// A message-passing network over the stored entries (edges) of A produces
// the values of M on A's pattern (the network is defined in spai.h).  The
// three message layers are dense contractions, [edges x 96] x [96 x 32]
// forward and [edges x 32] x [32 x 96] plus the weight gradient
// [32 x edges] x [edges x 96] backward, and run on the matrix cores with
// v_mfma_f32_32x32x16_bf16: one wave per 32-edge tile, bfloat16 operands,
// float32 accumulation.  Node and edge states are float32 in memory and
// enter the matrix cores as a pair of bfloat16 values (hi + lo, about 16
// significant bits) against weights that are exact in bfloat16: rounding
// the activations to one bfloat16 flips relu decisions near zero and, with
// the cancellation in the encoder-weight sums, costs several per cent of
// gradient accuracy.  Everything else is plain float32 vector code.  Every reduction is
// a fixed-order sum of per-wave or per-block partial rows: results do not
// depend on scheduling.
#include <math.h>

#include <algorithm>

#include "spai_internal.hpp"

namespace sp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// float32 -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// 8 consecutive float32 values as bfloat16 pairs: hi = bf16(v), lo = bf16(v - hi)
__device__ __forceinline__ void f8_split(const float* p, u16x8& hi, u16x8& lo) {
  const f32x4 a = *reinterpret_cast<const f32x4*>(p);
  const f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float v = q < 4 ? a[q] : b[q - 4];
    hi[q] = f2bf(v);
    lo[q] = f2bf(v - bf2f(hi[q]));
  }
}

// Operand fragment kb (0..5) of the message input u_e = [h_i, h_j, e_e] for
// the lane that owns edge e: the 8 features 16 kb + 8 half .. + 8.
__device__ __forceinline__ void u_frag(const float* __restrict__ hprev, const float* __restrict__ eprev, int i,
                                       int j, int e, int kb, int half, u16x8& hi, u16x8& lo) {
  const int f0 = 16 * (kb & 1) + 8 * half;
  const float* p = kb < 2 ? hprev + (size_t)i * kH : (kb < 4 ? hprev + (size_t)j * kH : eprev + (size_t)e * kH);
  f8_split(p + f0, hi, lo);
}

// output row (edge or feature) of accumulator r for lanes of `half`
__device__ __forceinline__ int acc_row(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }

// ------------------------------------------------------------ inputs
__global__ void k_diag(Net a, const double* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double aii = 0.0;
  for (int e = a.rp[i]; e < a.rp[i + 1]; ++e)
    if (a.ci[e] == i) aii = vals[e];
  const double d = aii != 0.0 ? fabs(aii) : 1.0;
  a.dis[i] = (float)(1.0 / sqrt(d));
  a.sig[i] = aii < 0.0 ? -1.0f : 1.0f;
}

__global__ void k_edges(Net a, const double* __restrict__ vals) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nnz) return;
  const double v = vals[e];
  a.ahat[e] = (float)(v * (double)a.dis[a.erow[e]] * (double)a.dis[a.ci[e]]);
  a.a32[e] = (float)v;
}

__global__ void k_xnode(Net a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
    if (a.ci[e] == i) continue;
    s0 += a.ahat[e];
    s1 += fabsf(a.ahat[e]);
  }
  for (int q = a.cp[i]; q < a.cp[i + 1]; ++q) {
    const int e = a.ce[q];
    if (a.erow[e] != i) s2 += a.ahat[e];
  }
  a.x[(size_t)i * 4 + 0] = s0;
  a.x[(size_t)i * 4 + 1] = s1;
  a.x[(size_t)i * 4 + 2] = s2;
  a.x[(size_t)i * 4 + 3] = 0.f;
}

__device__ __forceinline__ void edge_input(const Net& a, int e, float f[3]) {
  const int t = a.tpos[e];
  f[0] = a.ahat[e];
  f[1] = t >= 0 ? a.ahat[t] : 0.f;
  f[2] = a.erow[e] == a.ci[e] ? 1.f : 0.f;
}

// ------------------------------------------------------------ forward
__global__ void k_enc_node(Net a, const uint16_t* __restrict__ prm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.n * kH) return;
  const int i = (int)(idx / kH), f = (int)(idx % kH);
  float pre = bf2f(prm[obn + f]);
  for (int k = 0; k < kNin; ++k) pre += bf2f(prm[oWn + f * kNin + k]) * a.x[(size_t)i * 4 + k];
  a.h[0][idx] = fmaxf(pre, 0.f);
}

__global__ void k_enc_edge(Net a, const uint16_t* __restrict__ prm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.nnz * kH) return;
  const int e = (int)(idx / kH), f = (int)(idx % kH);
  float in[3];
  edge_input(a, e, in);
  float pre = bf2f(prm[obe + f]);
  for (int k = 0; k < kNin; ++k) pre += bf2f(prm[oWe + f * kNin + k]) * in[k];
  a.e[0][idx] = fmaxf(pre, 0.f);
}

// m_e = relu(W_L u_e + b_L) on the matrix cores: tile groups of 4 tiles per
// block (one tile per wave), grid-strided.
template <int L>
__global__ __launch_bounds__(256) void k_msg_fwd(Net a, const uint16_t* __restrict__ prm) {
  const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
  const uint16_t* W = prm + oW(L);
  bf16x8 B[6];
#pragma unroll
  for (int kb = 0; kb < 6; ++kb)
    B[kb] = as_bf(*reinterpret_cast<const u16x8*>(W + col * kU + 16 * kb + 8 * half));
  const float bias = bf2f(prm[ob(L) + col]);
  const float* hprev = a.h[L - 1];
  const float* eprev = a.e[L - 1];
  float* enext = a.e[L];
  const int ngroups = (a.ntile + kWavesPerBlock - 1) / kWavesPerBlock;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int t = g * kWavesPerBlock + wib;
    if (t >= a.ntile) continue;
    const int e = t * kEdgeTile + col;
    const bool ok = e < a.nnz;
    const int i = ok ? a.erow[e] : 0, j = ok ? a.ci[e] : 0;
    f32x16 acc = {};
#pragma unroll
    for (int kb = 0; kb < 6; ++kb) {
      u16x8 hi = {}, lo = {};
      if (ok) u_frag(hprev, eprev, i, j, e, kb, half, hi, lo);
      acc = mfma32(as_bf(hi), B[kb], acc);
      acc = mfma32(as_bf(lo), B[kb], acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ee = t * kEdgeTile + acc_row(r, half);
      if (ee < a.nnz) enext[(size_t)ee * kH + col] = fmaxf(acc[r] + bias, 0.f);
    }
  }
}

// h_L = h_{L-1} + (1/deg_i) sum_{e in row i} m_e
template <int L>
__global__ void k_agg(Net a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.n * kH) return;
  const int i = (int)(idx / kH), f = (int)(idx % kH);
  const int p0 = a.rp[i], p1 = a.rp[i + 1];
  float s = 0.f;
  for (int e = p0; e < p1; ++e) s += a.e[L][(size_t)e * kH + f];
  a.h[L][idx] = a.h[L - 1][idx] + (p1 > p0 ? s / (float)(p1 - p0) : 0.f);
}

// s_e = wo . [h_i, h_j, e_e] + bo, M_e = (sigma_i [i == j] + s_e) / sqrt(d_i d_j):
// 32 lanes per edge, one feature each.
__global__ void k_dec(Net a, const uint16_t* __restrict__ prm, float* __restrict__ mout) {
  const int e = blockIdx.x * 8 + (threadIdx.x >> 5);
  const int f = threadIdx.x & 31;
  const bool ok = e < a.nnz;
  const int i = ok ? a.erow[e] : 0, j = ok ? a.ci[e] : 0;
  float v = 0.f;
  if (ok)
    v = bf2f(prm[owo + f]) * a.h[3][(size_t)i * kH + f] + bf2f(prm[owo + kH + f]) * a.h[3][(size_t)j * kH + f] +
        bf2f(prm[owo + 2 * kH + f]) * a.e[3][(size_t)e * kH + f];
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (ok && f == 0) {
    const float s = v + bf2f(prm[obo]);
    mout[e] = ((i == j ? a.sig[i] : 0.f) + s) * a.dis[i] * a.dis[j];
  }
}

// ------------------------------------------------------------ loss
// Y_k = M Z_k (grid.y = k)
__global__ void k_spmv_m(Net a, const float* __restrict__ mv, const float* __restrict__ Z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const size_t o = (size_t)blockIdx.y * a.n;
  float s = 0.f;
  for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) s += mv[e] * Z[o + a.ci[e]];
  a.kbuf[o + i] = s;
}

__device__ double block_sum_d(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sh[q];
  return s;
}

// R_k = A Y_k - Z_k, partial sums of ||R_k||^2 and ||Z_k||^2 per block
__global__ void k_spmv_res(Net a, const float* __restrict__ Z, int nblk) {
  __shared__ double sh[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const size_t o = (size_t)k * a.n;
  const float* Y = a.kbuf;
  float* R = a.kbuf + (size_t)a.K * a.n;
  double rr = 0.0, zz = 0.0;
  if (i < a.n) {
    float s = 0.f;
    for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) s += a.a32[e] * Y[o + a.ci[e]];
    const float z = Z[o + i];
    const float r = s - z;
    R[o + i] = r;
    rr = (double)r * r;
    zz = (double)z * z;
  }
  rr = block_sum_d(rr, sh);
  zz = block_sum_d(zz, sh);
  if (threadIdx.x == 0) {
    a.lpart[(size_t)k * nblk + blockIdx.x] = rr;
    a.lpart[(size_t)(a.K + k) * nblk + blockIdx.x] = zz;
  }
}

// G_k = A^T R_k through the transposed pattern (fixed order per column)
__global__ void k_spmv_at(Net a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const size_t o = (size_t)blockIdx.y * a.n;
  const float* R = a.kbuf + (size_t)a.K * a.n;
  float* G = a.kbuf + (size_t)2 * a.K * a.n;
  float s = 0.f;
  for (int q = a.cp[j]; q < a.cp[j + 1]; ++q) {
    const int e = a.ce[q];
    s += a.a32[e] * R[o + a.erow[e]];
  }
  G[o + j] = s;
}

__global__ void k_loss_fin(Net a, int nblk) {
  __shared__ double sh[4];
  __shared__ double rr[64], zz[64];
  for (int k = 0; k < a.K; ++k) {
    double r = 0.0, z = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
      r += a.lpart[(size_t)k * nblk + b];
      z += a.lpart[(size_t)(a.K + k) * nblk + b];
    }
    r = block_sum_d(r, sh);
    z = block_sum_d(z, sh);
    if (threadIdx.x == 0) {
      rr[k] = r;
      zz[k] = z;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L = 0.0;
    int bad = 0;
    for (int k = 0; k < a.K; ++k) {
      if (!(zz[k] > 0.0)) {
        bad = 1;
        a.coef[k] = 0.f;
        continue;
      }
      L += rr[k] / zz[k];
      a.coef[k] = (float)(2.0 / ((double)a.K * zz[k]));
    }
    a.lossv[0] = L / a.K;
    a.bad[0] = bad;
  }
}

// dL/dM_e = sum_k coef_k G_k[i] Z_k[j]
__global__ void k_dm(Net a, const float* __restrict__ Z, float* __restrict__ dm) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nnz) return;
  const float* G = a.kbuf + (size_t)2 * a.K * a.n;
  const int i = a.erow[e], j = a.ci[e];
  float s = 0.f;
  for (int k = 0; k < a.K; ++k) s += a.coef[k] * G[(size_t)k * a.n + i] * Z[(size_t)k * a.n + j];
  dm[e] = s;
}

// ------------------------------------------------------------ backward
__global__ void k_ds(Net a, const float* __restrict__ dm) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nnz) return;
  a.ds[e] = dm[e] * a.dis[a.erow[e]] * a.dis[a.ci[e]];
}

// Sums sh[q][c] over the 8 slots q in order; 32 columns per row.
__device__ __forceinline__ float slot_sum(float (*sh)[kH + 1], int c) {
  float s = 0.f;
  for (int q = 0; q < 8; ++q) s += sh[q][c];
  return s;
}

// Decoder, edge part: de3_e = ds_e wo[64:96]; partials of sum_e ds_e e3_e and sum_e ds_e.
__global__ void k_dec_bwd_edge(Net a, const uint16_t* __restrict__ prm) {
  __shared__ float sh[8][kH + 1];
  const int q = threadIdx.x >> 5, f = threadIdx.x & 31;
  const float w = bf2f(prm[owo + 2 * kH + f]);
  float accw = 0.f, accb = 0.f;
  for (int e = blockIdx.x * 8 + q; e < a.nnz; e += gridDim.x * 8) {
    const float d = a.ds[e];
    a.de[(size_t)e * kH + f] = d * w;
    accw += d * a.e[3][(size_t)e * kH + f];
    if (f == 0) accb += d;
  }
  sh[q][f] = accw;
  if (f == 0) sh[q][kH] = accb;
  __syncthreads();
  float* P = a.part + (size_t)blockIdx.x * kDecEdgePart;
  if (threadIdx.x < kH) P[threadIdx.x] = slot_sum(sh, threadIdx.x);
  if (threadIdx.x == kH) P[kH] = slot_sum(sh, kH);
}

// Decoder, node part: dh3_i = (sum_{row i} ds) wo[0:32] + (sum_{col i} ds) wo[32:64];
// partials of sum_i rowsum_i h3_i and sum_i colsum_i h3_i.
__global__ void k_dec_bwd_node(Net a, const uint16_t* __restrict__ prm) {
  __shared__ float sh1[8][kH + 1], sh2[8][kH + 1];
  const int q = threadIdx.x >> 5, f = threadIdx.x & 31;
  const float w1 = bf2f(prm[owo + f]), w2 = bf2f(prm[owo + kH + f]);
  float acc1 = 0.f, acc2 = 0.f;
  for (int i = blockIdx.x * 8 + q; i < a.n; i += gridDim.x * 8) {
    float rs = 0.f, cs = 0.f;
    for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) rs += a.ds[e];
    for (int p = a.cp[i]; p < a.cp[i + 1]; ++p) cs += a.ds[a.ce[p]];
    a.dh[0][(size_t)i * kH + f] = rs * w1 + cs * w2;
    const float hv = a.h[3][(size_t)i * kH + f];
    acc1 += rs * hv;
    acc2 += cs * hv;
  }
  sh1[q][f] = acc1;
  sh2[q][f] = acc2;
  __syncthreads();
  float* P = a.part + (size_t)blockIdx.x * kDecNodePart;
  if (threadIdx.x < kH) P[threadIdx.x] = slot_sum(sh1, threadIdx.x);
  else if (threadIdx.x < 2 * kH) P[threadIdx.x] = slot_sum(sh2, threadIdx.x - kH);
}

// Message layer L backward on the matrix cores.  Per 32-edge tile (one wave):
//   dm = de_L + dh_L[i] / deg_i, dpre = dm * [m > 0]
//   du = dpre W_L -> (per edge) towards h_i, towards h_j, and de_{L-1} (in place),
//        with dpre split into two bfloat16 terms
//   dW_L += dpre^T u, db_L += sum dpre   (per-wave partial rows; both
//   operands split, hi*hi + lo*hi + hi*lo: the sum over edges cancels
//   strongly, so single-bfloat16 operands would cost ~1e-2 relative)
template <int L>
__global__ __launch_bounds__(256) void k_msg_bwd(Net a, const uint16_t* __restrict__ prm,
                                                 const float* __restrict__ dhin) {
  // float32 tiles of u and dpre per wave; the db reduction reuses the u tiles
  __shared__ __align__(16) float ulds[kWavesPerBlock][kEdgeTile][kU];
  __shared__ __align__(16) float dlds[kWavesPerBlock][kEdgeTile][kH];
  float(*dbl)[64][17] = reinterpret_cast<float(*)[64][17]>(&ulds[0][0][0]);
  static_assert(sizeof(float) * kWavesPerBlock * 64 * 17 <= sizeof(float) * kWavesPerBlock * kEdgeTile * kU, "");
  const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  const uint16_t* W = prm + oW(L);
  bf16x8 Bd[2][3];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int nt = 0; nt < 3; ++nt) {
      u16x8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = W[(16 * kb + 8 * half + q) * kU + 32 * nt + col];
      Bd[kb][nt] = as_bf(v);
    }
  f32x16 dW[3] = {};
  float dbacc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) dbacc[q] = 0.f;
  const float* hprev = a.h[L - 1];
  const float* eprev = a.e[L - 1];
  const float* ecur = a.e[L];
  const int ngroups = (a.ntile + kWavesPerBlock - 1) / kWavesPerBlock;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {  // uniform trip count per block
    const int t = g * kWavesPerBlock + wib;
    const int e = t * kEdgeTile + col;
    const bool ok = t < a.ntile && e < a.nnz;
    int i = 0, j = 0;
    float inv = 0.f;
    if (ok) {
      i = a.erow[e];
      j = a.ci[e];
      inv = 1.f / (float)(a.rp[i + 1] - a.rp[i]);
    }
#pragma unroll
    for (int kb = 0; kb < 6; ++kb) {
      const int f0 = 16 * (kb & 1) + 8 * half;
      f32x4 v0 = {}, v1 = {};
      if (ok) {
        const float* p = kb < 2 ? hprev + (size_t)i * kH : (kb < 4 ? hprev + (size_t)j * kH : eprev + (size_t)e * kH);
        v0 = *reinterpret_cast<const f32x4*>(p + f0);
        v1 = *reinterpret_cast<const f32x4*>(p + f0 + 4);
      }
      *reinterpret_cast<f32x4*>(&ulds[wib][col][16 * kb + 8 * half]) = v0;
      *reinterpret_cast<f32x4*>(&ulds[wib][col][16 * kb + 8 * half + 4]) = v1;
    }
    // dpre as a pair of bfloat16 values (hi + lo): the weights are exact in
    // bfloat16, so du = dpre W keeps about 16 significant bits through the
    // layers; the weight gradient uses hi only
    bf16x8 Ad[2], Al[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int f0 = 16 * kb + 8 * half;
      u16x8 dv = {}, dl = {};
      float dps[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (ok) {
        const f32x4 d0 = *reinterpret_cast<const f32x4*>(a.de + (size_t)e * kH + f0);
        const f32x4 d1 = *reinterpret_cast<const f32x4*>(a.de + (size_t)e * kH + f0 + 4);
        const f32x4 h0 = *reinterpret_cast<const f32x4*>(dhin + (size_t)i * kH + f0);
        const f32x4 h1 = *reinterpret_cast<const f32x4*>(dhin + (size_t)i * kH + f0 + 4);
        const f32x4 m0 = *reinterpret_cast<const f32x4*>(ecur + (size_t)e * kH + f0);
        const f32x4 m1 = *reinterpret_cast<const f32x4*>(ecur + (size_t)e * kH + f0 + 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float dm = (q < 4 ? d0[q] : d1[q - 4]) + (q < 4 ? h0[q] : h1[q - 4]) * inv;
          const float dp = (q < 4 ? m0[q] : m1[q - 4]) > 0.f ? dm : 0.f;
          dbacc[8 * kb + q] += dp;
          dps[q] = dp;
          dv[q] = f2bf(dp);
          dl[q] = f2bf(dp - bf2f(dv[q]));
        }
      }
      Ad[kb] = as_bf(dv);
      Al[kb] = as_bf(dl);
      *reinterpret_cast<f32x4*>(&dlds[wib][col][f0]) = f32x4{dps[0], dps[1], dps[2], dps[3]};
      *reinterpret_cast<f32x4*>(&dlds[wib][col][f0 + 4]) = f32x4{dps[4], dps[5], dps[6], dps[7]};
    }
    f32x16 du[3] = {};
#pragma unroll
    for (int nt = 0; nt < 3; ++nt)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        du[nt] = mfma32(Ad[kb], Bd[kb][nt], du[nt]);
        du[nt] = mfma32(Al[kb], Bd[kb][nt], du[nt]);
      }
    if (t < a.ntile) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ee = t * kEdgeTile + acc_row(r, half);
        if (ee < a.nnz) {
          a.duhi[(size_t)ee * kH + col] = du[0][r];
          a.duhj[(size_t)ee * kH + col] = du[1][r];
          a.de[(size_t)ee * kH + col] = du[2][r];
        }
      }
    }
    __syncthreads();  // the tile's u and dpre are in LDS
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      u16x8 ah, al;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float v = dlds[wib][16 * kb + 8 * half + q][col];
        ah[q] = f2bf(v);
        al[q] = f2bf(v - bf2f(ah[q]));
      }
#pragma unroll
      for (int nt = 0; nt < 3; ++nt) {
        u16x8 bh, bl;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float v = ulds[wib][16 * kb + 8 * half + q][32 * nt + col];
          bh[q] = f2bf(v);
          bl[q] = f2bf(v - bf2f(bh[q]));
        }
        dW[nt] = mfma32(as_bf(ah), as_bf(bh), dW[nt]);
        dW[nt] = mfma32(as_bf(al), as_bf(bh), dW[nt]);
        dW[nt] = mfma32(as_bf(ah), as_bf(bl), dW[nt]);
      }
    }
    __syncthreads();  // LDS is rewritten by the next tile
  }
  float* P = a.part + (size_t)wave * kLayerPart;
#pragma unroll
  for (int nt = 0; nt < 3; ++nt)
#pragma unroll
    for (int r = 0; r < 16; ++r) P[acc_row(r, half) * kU + 32 * nt + col] = dW[nt][r];
#pragma unroll
  for (int q = 0; q < 16; ++q) dbl[wib][lane][q] = dbacc[q];
  __syncthreads();
  if (lane < kH) {  // feature ff = 16 kb + 8 hf + q, held by the lanes of half hf
    const int kb = lane >> 4, hf = (lane >> 3) & 1, q = lane & 7;
    float s = 0.f;
    for (int c = 0; c < 32; ++c) s += dbl[wib][hf * 32 + c][8 * kb + q];
    P[kH * kU + lane] = s;
  }
}

// dh_{L-1}[i] = dh_L[i] + sum_{row i} du_hi + sum_{col i} du_hj
__global__ void k_node_bwd(Net a, const float* __restrict__ dhin, float* __restrict__ dhout) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.n * kH) return;
  const int i = (int)(idx / kH), f = (int)(idx % kH);
  float s = dhin[idx];
  for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) s += a.duhi[(size_t)e * kH + f];
  for (int p = a.cp[i]; p < a.cp[i + 1]; ++p) s += a.duhj[(size_t)a.ce[p] * kH + f];
  dhout[idx] = s;
}

// Encoders backward: partials of dWn / dbn (nodes) and dWe / dbe (edges).
__global__ void k_enc_bwd_node(Net a, const float* __restrict__ dh0) {
  __shared__ float sh[4][8][kH + 1];
  const int q = threadIdx.x >> 5, f = threadIdx.x & 31;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int i = blockIdx.x * 8 + q; i < a.n; i += gridDim.x * 8) {
    const size_t o = (size_t)i * kH + f;
    const float dp = a.h[0][o] > 0.f ? dh0[o] : 0.f;
    for (int k = 0; k < kNin; ++k) acc[k] += dp * a.x[(size_t)i * 4 + k];
    acc[3] += dp;
  }
  for (int k = 0; k < 4; ++k) sh[k][q][f] = acc[k];
  __syncthreads();
  float* P = a.part + (size_t)blockIdx.x * kEncPart;
  if (threadIdx.x < kH) {
    const int ff = threadIdx.x;
    for (int k = 0; k < kNin; ++k) P[ff * kNin + k] = slot_sum(sh[k], ff);
    P[kH * kNin + ff] = slot_sum(sh[3], ff);
  }
}

__global__ void k_enc_bwd_edge(Net a) {
  __shared__ float sh[4][8][kH + 1];
  const int q = threadIdx.x >> 5, f = threadIdx.x & 31;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int e = blockIdx.x * 8 + q; e < a.nnz; e += gridDim.x * 8) {
    const size_t o = (size_t)e * kH + f;
    const float dp = a.e[0][o] > 0.f ? a.de[o] : 0.f;
    float in[3];
    edge_input(a, e, in);
    for (int k = 0; k < kNin; ++k) acc[k] += dp * in[k];
    acc[3] += dp;
  }
  for (int k = 0; k < 4; ++k) sh[k][q][f] = acc[k];
  __syncthreads();
  float* P = a.part + (size_t)blockIdx.x * kEncPart;
  if (threadIdx.x < kH) {
    const int ff = threadIdx.x;
    for (int k = 0; k < kNin; ++k) P[ff * kNin + k] = slot_sum(sh[k], ff);
    P[kH * kNin + ff] = slot_sum(sh[3], ff);
  }
}

// grad[dst + c] (=, or +=) the sum over rows b of part[b * stride + src + c]:
// a block covers 32 columns with 8 row groups; group g sums the rows
// b = g mod 8 in order, then the 8 group sums are added in order.
__global__ void k_reduce(const float* __restrict__ part, int rows, int stride, int src, int count,
                         float* __restrict__ grad, int dst, int accumulate) {
  __shared__ double sh[8][33];
  const int cl = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cl;
  double s = 0.0;
  if (c < count)
    for (int b = g; b < rows; b += 8) s += (double)part[(size_t)b * stride + src + c];
  sh[g][cl] = s;
  __syncthreads();
  if (g == 0 && c < count) {
    double t = 0.0;
    for (int q = 0; q < 8; ++q) t += sh[q][cl];
    grad[dst + c] = accumulate ? grad[dst + c] + (float)t : (float)t;
  }
}

__global__ void k_flag_clear(int32_t* flag) { flag[0] = 0; }

// sets flag when an entry of (row_ptr, col_idx) differs from the pattern
__global__ void k_compare_pattern(Net a, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool diff = false;
  if (k <= a.n) diff = rp[k] != a.rp[k];
  if (k < a.nnz) diff = diff || ci[k] != a.ci[k];
  if (diff) a.bad[0] = 1;
}

__global__ void k_adam(int64_t count, float* __restrict__ theta, uint16_t* __restrict__ pb,
                       const float* __restrict__ grad, float gscale, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const float g = grad[k] * gscale;
  const float a1 = b1 * m1[k] + (1.f - b1) * g;
  const float a2 = b2 * m2[k] + (1.f - b2) * g * g;
  m1[k] = a1;
  m2[k] = a2;
  const float th = theta[k] - lr * (a1 / c1) / (sqrtf(a2 / c2) + eps);
  theta[k] = th;
  pb[k] = f2bf(th);
}

int grid_for(int64_t threads) { return (int)((threads + 255) / 256); }

int mfma_blocks(const Net& a, int ncu) {
  const int groups = (a.ntile + kWavesPerBlock - 1) / kWavesPerBlock;
  return std::max(1, std::min(2 * ncu, groups));
}

int small_blocks(int ncu) { return std::max(1, 2 * ncu); }

}  // namespace

int loss_blocks(int n) { return grid_for(n); }

size_t backward_part_floats(int n, int nnz, int ncu) {
  (void)n;
  Net t{};
  t.nnz = nnz;
  t.ntile = (nnz + kEdgeTile - 1) / kEdgeTile;
  const size_t mf = (size_t)mfma_blocks(t, ncu) * kWavesPerBlock * kLayerPart;
  const size_t sm = (size_t)small_blocks(ncu) * std::max(std::max(kDecEdgePart, kDecNodePart), kEncPart);
  return std::max(mf, sm);
}

hipError_t launch_features(const Net& a, const double* vals, hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3(grid_for(a.n)), dim3(256), 0, st, a, vals);
  hipLaunchKernelGGL(k_edges, dim3(grid_for(a.nnz)), dim3(256), 0, st, a, vals);
  hipLaunchKernelGGL(k_xnode, dim3(grid_for(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_forward(const Net& a, const uint16_t* prm, float* m_out, int ncu, hipStream_t st) {
  hipLaunchKernelGGL(k_enc_node, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a, prm);
  hipLaunchKernelGGL(k_enc_edge, dim3(grid_for((int64_t)a.nnz * kH)), dim3(256), 0, st, a, prm);
  const int gm = mfma_blocks(a, ncu);
  hipLaunchKernelGGL(k_msg_fwd<1>, dim3(gm), dim3(256), 0, st, a, prm);
  hipLaunchKernelGGL(k_agg<1>, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_msg_fwd<2>, dim3(gm), dim3(256), 0, st, a, prm);
  hipLaunchKernelGGL(k_agg<2>, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_msg_fwd<3>, dim3(gm), dim3(256), 0, st, a, prm);
  hipLaunchKernelGGL(k_agg<3>, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_dec, dim3((a.nnz + 7) / 8), dim3(256), 0, st, a, prm, m_out);
  return hipGetLastError();
}

hipError_t launch_loss(const Net& a, const float* mv, const float* Z, int nblk, float* dm, hipStream_t st) {
  const dim3 g((unsigned)nblk, (unsigned)a.K);
  hipLaunchKernelGGL(k_spmv_m, g, dim3(256), 0, st, a, mv, Z);
  hipLaunchKernelGGL(k_spmv_res, g, dim3(256), 0, st, a, Z, nblk);
  hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(256), 0, st, a, nblk);
  if (dm) {
    hipLaunchKernelGGL(k_spmv_at, g, dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_dm, dim3(grid_for(a.nnz)), dim3(256), 0, st, a, Z, dm);
  }
  return hipGetLastError();
}

hipError_t launch_backward(const Net& a, const uint16_t* prm, const float* dm, float* grad, int accumulate,
                           int ncu, hipStream_t st) {
  const int gs = small_blocks(ncu);
  const int gm = mfma_blocks(a, ncu);
  const int acc = accumulate ? 1 : 0;
  auto reduce = [&](int rows, int stride, int src, int count, int dst) {
    hipLaunchKernelGGL(k_reduce, dim3((count + 31) / 32), dim3(256), 0, st, a.part, rows, stride, src, count, grad,
                       dst, acc);
  };
  hipLaunchKernelGGL(k_ds, dim3(grid_for(a.nnz)), dim3(256), 0, st, a, dm);
  hipLaunchKernelGGL(k_dec_bwd_edge, dim3(gs), dim3(256), 0, st, a, prm);
  reduce(gs, kDecEdgePart, 0, kH, owo + 2 * kH);
  reduce(gs, kDecEdgePart, kH, 1, obo);
  hipLaunchKernelGGL(k_dec_bwd_node, dim3(gs), dim3(256), 0, st, a, prm);
  reduce(gs, kDecNodePart, 0, 2 * kH, owo);
  // dh_3 is in dh[0]; layers alternate the two node-gradient buffers
  hipLaunchKernelGGL(k_msg_bwd<3>, dim3(gm), dim3(256), 0, st, a, prm, a.dh[0]);
  reduce(gm * kWavesPerBlock, kLayerPart, 0, kH * kU, oW3);
  reduce(gm * kWavesPerBlock, kLayerPart, kH * kU, kH, ob3);
  hipLaunchKernelGGL(k_node_bwd, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a, a.dh[0], a.dh[1]);
  hipLaunchKernelGGL(k_msg_bwd<2>, dim3(gm), dim3(256), 0, st, a, prm, a.dh[1]);
  reduce(gm * kWavesPerBlock, kLayerPart, 0, kH * kU, oW2);
  reduce(gm * kWavesPerBlock, kLayerPart, kH * kU, kH, ob2);
  hipLaunchKernelGGL(k_node_bwd, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a, a.dh[1], a.dh[0]);
  hipLaunchKernelGGL(k_msg_bwd<1>, dim3(gm), dim3(256), 0, st, a, prm, a.dh[0]);
  reduce(gm * kWavesPerBlock, kLayerPart, 0, kH * kU, oW1);
  reduce(gm * kWavesPerBlock, kLayerPart, kH * kU, kH, ob1);
  hipLaunchKernelGGL(k_node_bwd, dim3(grid_for((int64_t)a.n * kH)), dim3(256), 0, st, a, a.dh[0], a.dh[1]);
  hipLaunchKernelGGL(k_enc_bwd_node, dim3(gs), dim3(256), 0, st, a, a.dh[1]);
  reduce(gs, kEncPart, 0, kH * kNin, oWn);
  reduce(gs, kEncPart, kH * kNin, kH, obn);
  hipLaunchKernelGGL(k_enc_bwd_edge, dim3(gs), dim3(256), 0, st, a);
  reduce(gs, kEncPart, 0, kH * kNin, oWe);
  reduce(gs, kEncPart, kH * kNin, kH, obe);
  return hipGetLastError();
}

hipError_t launch_compare_pattern(const Net& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, st, a.bad);
  hipLaunchKernelGGL(k_compare_pattern, dim3(grid_for(std::max<int64_t>(a.n + 1, a.nnz))), dim3(256), 0, st, a,
                     row_ptr, col_idx);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* theta, uint16_t* pb, const float* grad, float gscale, float* m1,
                       float* m2, float lr, float b1, float b2, float eps, int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(count)), dim3(256), 0, st, count, theta, pb, grad, gscale, m1, m2, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace sp

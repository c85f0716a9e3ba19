// Internal declarations of the learned sparse approximate inverse (network
// kernels and their host driver).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp {

constexpr int kH = 32;    // hidden width
constexpr int kU = 96;    // message input width [h_i, h_j, e_ij]
constexpr int kNin = 3;   // node / edge input features
constexpr int kNParams = 9665;
constexpr int kEdgeTile = 32;  // edges per matrix-core tile (one wave)
constexpr int kWavesPerBlock = 4;

// flat parameter layout (matrices row-major, output x input)
constexpr int oWn = 0, obn = 96, oWe = 128, obe = 224;
constexpr int oW1 = 256, ob1 = 3328, oW2 = 3360, ob2 = 6432, oW3 = 6464, ob3 = 9536;
constexpr int owo = 9568, obo = 9664;
__host__ __device__ constexpr int oW(int l) { return l == 1 ? oW1 : (l == 2 ? oW2 : oW3); }
__host__ __device__ constexpr int ob(int l) { return l == 1 ? ob1 : (l == 2 ? ob2 : ob3); }

// per-wave partial row of a message layer's weight gradient: W (32 x 96), b (32)
constexpr int kLayerPart = kH * kU + kH;
// per-block partial rows of the small reductions
constexpr int kDecEdgePart = kH + 1;  // wo[64:96], bo
constexpr int kDecNodePart = 2 * kH;  // wo[0:32], wo[32:64]
constexpr int kEncPart = kH * kNin + kH;

struct Net {
  int32_t n, nnz, ntile;  // ntile = edge tiles of kEdgeTile
  int32_t K;              // residual vectors of the current loss call
  const int32_t* rp;      // CSR row pointer [n + 1]
  const int32_t* ci;      // column of each edge [nnz]
  const int32_t* erow;    // row of each edge [nnz]
  const int32_t* tpos;    // edge index of the transposed entry, -1 if not stored
  const int32_t* cp;      // transposed pattern: edges of column j are ce[cp[j] .. cp[j+1])
  const int32_t* ce;      //   (ascending edge index)
  float* ahat;            // a_ij / sqrt(d_i d_j)
  float* dis;             // 1 / sqrt(d_i)
  float* sig;             // sign of a_ii (1 if zero)
  float* a32;             // float32 values of A
  float* x;               // node inputs [n][4] (last one unused)
  float* h[4];            // node states after the encoder and each layer [n][32]
  float* e[4];            // edge states [nnz][32]
  float* dh[2];           // node gradients (ping-pong) [n][32]
  float* de;              // edge gradients [nnz][32]
  float* duhi;            // per-edge gradient towards h_i [nnz][32]
  float* duhj;            // per-edge gradient towards h_j [nnz][32]
  float* ds;              // gradient of the decoder output [nnz]
  float* part;            // parameter-gradient partial rows
  double* lpart;          // loss partials [2][kmax][nblk]
  float* kbuf;            // loss work vectors: Y, R, G [3][kmax][n]
  float* coef;            // [kmax] 2 / (K ||z_k||^2)
  double* lossv;          // [1] loss
  int32_t* bad;           // [1] a zero residual vector was passed
};

// launchers (all enqueue on `st` and return hipGetLastError())
hipError_t launch_features(const Net& a, const double* vals, hipStream_t st);
hipError_t launch_forward(const Net& a, const uint16_t* prm, float* m_out, int ncu, hipStream_t st);
hipError_t launch_loss(const Net& a, const float* mv, const float* Z, int nblk, float* dm, hipStream_t st);
hipError_t launch_backward(const Net& a, const uint16_t* prm, const float* dm, float* grad, int accumulate,
                           int ncu, hipStream_t st);
// a.bad = 0 if (row_ptr, col_idx) equal the network's pattern, else 1
hipError_t launch_compare_pattern(const Net& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t st);
hipError_t launch_adam(int64_t count, float* theta, uint16_t* pb, const float* grad, float gscale, float* m1,
                       float* m2, float lr, float b1, float b2, float eps, int t, hipStream_t st);
// rows of the partial table the backward pass needs for `ncu` compute units
size_t backward_part_floats(int n, int nnz, int ncu);
int loss_blocks(int n);

}  // namespace sp

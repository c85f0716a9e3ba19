// gmres_encode_noalloc: the 2-byte basis encoding of gmres_encode with its
// partial maxima in a static device array instead of a buffer allocated per
// call, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "gmres.h"
#include "gmres_internal.hpp"

namespace {

// One partial maximum per 256-element tile (the tile of every other kernel
// of the library), then the maximum of those partials in slot 0.  The
// partials start 64 floats (256 bytes) in.
constexpr int64_t kMaxN = (int64_t)1 << 24;
constexpr int64_t kMaxTiles = kMaxN / gm::kTile;
constexpr int64_t kPartOffset = 64;

// Lives on every device the library runs on until the process ends.  In
// host code this name stands for the symbol, not for a device address: host
// code uses the per-device pointer from hipGetSymbolAddress below.
static __device__ __align__(256) float scratch[kPartOffset + kMaxTiles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_ptr(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMRES_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return GMRES_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return GMRES_EHIP;
    }
    g_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_ptr[dev];
  return GMRES_OK;
}

}  // namespace

extern "C" int gmres_encode_noalloc(int32_t precision, int64_t n, const float* w, double inv_h, void* out,
                                    double* scale_out, void* hip_stream) {
  if (precision != GMRES_MIXED_BF16 && precision != GMRES_MIXED_FP16) return GMRES_EINVAL;
  if (n < 0 || (n > 0 && (!w || !out)) || !(inv_h > 0.0)) return GMRES_EINVAL;
  if (n > kMaxN) return GMRES_EINVAL;  // more tiles than the static scratch holds
  float* ptr = nullptr;
  const int rc = scratch_ptr(&ptr);
  if (rc != GMRES_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  float mx = 0.0f;
  if (n > 0) {
    // per-tile maxima (every slot the reduction reads is written by this
    // call), then their maximum; the previous call's contents are never read
    const int ntiles = (int)((n + gm::kTile - 1) / gm::kTile);
    if (gm::launch_absmax(w, n, ptr + kPartOffset, ntiles, st) != hipSuccess ||
        gm::launch_absmax(ptr + kPartOffset, ntiles, ptr, 1, st) != hipSuccess ||
        hipMemcpyAsync(&mx, ptr, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      (void)hipGetLastError();
      return GMRES_EHIP;
    }
  }
  // the scale of gmres_encode: e with max|v| 2^e in (T/2, T]
  const double vmax = (double)mx * inv_h;
  int e = 0;
  if (vmax > 0.0 && std::isfinite(vmax)) {
    int p;
    const double f = std::frexp(vmax, &p);
    e = (precision == GMRES_MIXED_FP16 ? 15 : 0) - p + (f == 0.5 ? 1 : 0);
  }
  const float fac = (float)(std::ldexp(1.0, e) * inv_h);
  if (gm::launch_encode_plain(precision, n, w, fac, out, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return GMRES_EHIP;
  }
  if (scale_out) *scale_out = std::ldexp(1.0, -e);
  return GMRES_OK;
}

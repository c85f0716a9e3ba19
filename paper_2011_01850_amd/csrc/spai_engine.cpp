// Host side of the learned sparse approximate inverse: pattern preprocessing,
// device workspace, and the spai_* C-ABI of include/spai.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "spai.h"
#include "spai_internal.hpp"

namespace {

constexpr uint32_t kMagic = 0x5350414Au;  // "SPAJ"
constexpr int kMaxK = 64;

struct Fail {
  int code;
};

inline void hip_check(hipError_t e) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{GMRES_EHIP};
  }
}

}  // namespace

struct spai_ctx {
  uint32_t magic = kMagic;
  hipStream_t stream = nullptr;
  hipStream_t user = nullptr;
  hipEvent_t evu = nullptr;
  sp::Net a{};
  int kmax = 0, ncu = 1, nblk = 1;
  bool values_set = false, forward_done = false;
  bool loss_ready = false, backward_ready = false;  // workspaces allocated on first use
  std::vector<void*> allocs;

  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 256)) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{GMRES_ENOMEM};
    }
    allocs.push_back(p);
    return static_cast<T*>(p);
  }

  ~spai_ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : allocs) (void)hipFree(p);
    if (evu) (void)hipEventDestroy(evu);
    if (stream) (void)hipStreamDestroy(stream);
    magic = 0;
  }
};

namespace {

spai_ctx* get(spai_handle h) {
  if (!h || h->magic != kMagic) throw Fail{GMRES_EHANDLE};
  return h;
}

void after_caller(spai_ctx* h) {
  hip_check(hipEventRecord(h->evu, h->user));
  hip_check(hipStreamWaitEvent(h->stream, h->evu, 0));
}

template <typename T>
T* upload(spai_ctx* h, const std::vector<T>& v) {
  T* d = h->alloc<T>(v.size());
  if (!v.empty()) hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  return d;
}

void setup(spai_ctx* h, int64_t n64, int64_t nnz64, const int32_t* row_ptr, const int32_t* col_idx, int kmax,
           void* user_stream) {
  const int n = (int)n64, nnz = (int)nnz64;
  h->user = (hipStream_t)user_stream;
  h->kmax = kmax;
  hip_check(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  hip_check(hipEventCreateWithFlags(&h->evu, hipEventDisableTiming));
  after_caller(h);
  std::vector<int32_t> rp(n + 1), ci(nnz);
  hip_check(hipMemcpyAsync(rp.data(), row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  hip_check(hipMemcpyAsync(ci.data(), col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  hip_check(hipStreamSynchronize(h->stream));
  if (rp[0] != 0 || rp[n] != nnz) throw Fail{GMRES_EINVAL};
  for (int i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) throw Fail{GMRES_EINVAL};
  for (int e = 0; e < nnz; ++e)
    if (ci[e] < 0 || ci[e] >= n) throw Fail{GMRES_EINVAL};
  // row of each edge; per-row (column, edge) lists sorted by column for the
  // duplicate check and the transposed-entry lookup
  std::vector<int32_t> erow(nnz);
  std::vector<std::pair<int32_t, int32_t>> sorted(nnz);
  for (int i = 0; i < n; ++i) {
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      erow[e] = i;
      sorted[e] = {ci[e], e};
    }
    std::sort(sorted.begin() + rp[i], sorted.begin() + rp[i + 1]);
    for (int e = rp[i] + 1; e < rp[i + 1]; ++e)
      if (sorted[e].first == sorted[e - 1].first) throw Fail{GMRES_EINVAL};
  }
  std::vector<int32_t> tpos(nnz, -1);
  for (int e = 0; e < nnz; ++e) {
    const int i = erow[e], j = ci[e];
    auto b = sorted.begin() + rp[j], en = sorted.begin() + rp[j + 1];
    auto it = std::lower_bound(b, en, std::make_pair(i, (int32_t)-1));
    if (it != en && it->first == i) tpos[e] = it->second;
  }
  // transposed pattern: edges of each column in ascending edge order
  std::vector<int32_t> cp(n + 1, 0), ce(nnz);
  for (int e = 0; e < nnz; ++e) ++cp[ci[e] + 1];
  for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
  {
    std::vector<int32_t> fill(cp.begin(), cp.end() - 1);
    for (int e = 0; e < nnz; ++e) ce[fill[ci[e]]++] = e;
  }
  int dev = 0;
  hip_check(hipGetDevice(&dev));
  hip_check(hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, dev));
  h->nblk = sp::loss_blocks(n);
  sp::Net& a = h->a;
  a.n = n;
  a.nnz = nnz;
  a.ntile = (nnz + sp::kEdgeTile - 1) / sp::kEdgeTile;
  a.rp = upload(h, rp);
  a.ci = upload(h, ci);
  a.erow = upload(h, erow);
  a.tpos = upload(h, tpos);
  a.cp = upload(h, cp);
  a.ce = upload(h, ce);
  a.ahat = h->alloc<float>(nnz);
  a.dis = h->alloc<float>(n);
  a.sig = h->alloc<float>(n);
  a.a32 = h->alloc<float>(nnz);
  a.x = h->alloc<float>((size_t)n * 4);
  for (int l = 0; l < 4; ++l) {
    a.h[l] = h->alloc<float>((size_t)n * sp::kH);
    a.e[l] = h->alloc<float>((size_t)nnz * sp::kH);
  }
  hip_check(hipStreamSynchronize(h->stream));
}

void ensure_loss(spai_ctx* h) {
  if (h->loss_ready) return;
  sp::Net& a = h->a;
  a.lpart = h->alloc<double>((size_t)2 * h->kmax * h->nblk);
  a.kbuf = h->alloc<float>((size_t)3 * h->kmax * a.n);
  a.coef = h->alloc<float>(h->kmax);
  a.lossv = h->alloc<double>(1);
  a.bad = h->alloc<int32_t>(1);
  h->loss_ready = true;
}

void ensure_backward(spai_ctx* h) {
  if (h->backward_ready) return;
  sp::Net& a = h->a;
  a.dh[0] = h->alloc<float>((size_t)a.n * sp::kH);
  a.dh[1] = h->alloc<float>((size_t)a.n * sp::kH);
  a.de = h->alloc<float>((size_t)a.nnz * sp::kH);
  a.duhi = h->alloc<float>((size_t)a.nnz * sp::kH);
  a.duhj = h->alloc<float>((size_t)a.nnz * sp::kH);
  a.ds = h->alloc<float>(a.nnz);
  a.part = h->alloc<float>(sp::backward_part_floats(a.n, a.nnz, h->ncu));
  h->backward_ready = true;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Fail& x) {
    (void)hipGetLastError();
    return x.code;
  } catch (const std::bad_alloc&) {
    return GMRES_ENOMEM;
  }
}

}  // namespace

extern "C" {

int spai_create(spai_handle* out, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                int32_t kmax, void* hip_stream) {
  if (!out) return GMRES_EINVAL;
  *out = nullptr;
  if (n <= 0 || nnz <= 0 || n > INT32_MAX - 1 || nnz > INT32_MAX / sp::kH || !row_ptr || !col_idx || kmax < 1 ||
      kmax > kMaxK)
    return GMRES_EINVAL;
  spai_ctx* h = new (std::nothrow) spai_ctx();
  if (!h) return GMRES_ENOMEM;
  const int rc = guarded([&] {
    setup(h, n, nnz, row_ptr, col_idx, kmax, hip_stream);
    return GMRES_OK;
  });
  if (rc != GMRES_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return GMRES_OK;
}

int spai_set_values(spai_handle hh, const double* vals) {
  return guarded([&] {
    spai_ctx* h = get(hh);
    if (!vals) return GMRES_EINVAL;
    after_caller(h);
    hip_check(sp::launch_features(h->a, vals, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    h->values_set = true;
    h->forward_done = false;
    return GMRES_OK;
  });
}

int spai_forward(spai_handle hh, const uint16_t* params, float* m_out) {
  return guarded([&] {
    spai_ctx* h = get(hh);
    if (!params || !m_out) return GMRES_EINVAL;
    if (!h->values_set) return GMRES_ESTATE;
    after_caller(h);
    hip_check(sp::launch_forward(h->a, params, m_out, h->ncu, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    h->forward_done = true;
    return GMRES_OK;
  });
}

int spai_loss(spai_handle hh, const float* m_vals, const float* Z, int32_t K, double* loss_out, float* dm_out) {
  return guarded([&] {
    spai_ctx* h = get(hh);
    if (!m_vals || !Z || K < 1 || K > h->kmax) return GMRES_EINVAL;
    if (!h->values_set) return GMRES_ESTATE;
    ensure_loss(h);
    after_caller(h);
    sp::Net a = h->a;
    a.K = K;
    hip_check(sp::launch_loss(a, m_vals, Z, h->nblk, dm_out, h->stream));
    double L = 0.0;
    int32_t bad = 0;
    hip_check(hipMemcpyAsync(&L, a.lossv, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    hip_check(hipMemcpyAsync(&bad, a.bad, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    if (bad) return GMRES_EINVAL;
    if (loss_out) *loss_out = L;
    return GMRES_OK;
  });
}

int spai_backward(spai_handle hh, const uint16_t* params, const float* dm, float* grad, int32_t accumulate) {
  return guarded([&] {
    spai_ctx* h = get(hh);
    if (!params || !dm || !grad) return GMRES_EINVAL;
    if (!h->forward_done) return GMRES_ESTATE;
    ensure_backward(h);
    after_caller(h);
    hip_check(sp::launch_backward(h->a, params, dm, grad, accumulate, h->ncu, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    return GMRES_OK;
  });
}

int spai_same_pattern(spai_handle hh, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t* same_out) {
  return guarded([&] {
    spai_ctx* h = get(hh);
    if (!row_ptr || !col_idx || !same_out) return GMRES_EINVAL;
    if (n != h->a.n || nnz != h->a.nnz) {
      *same_out = 0;
      return GMRES_OK;
    }
    ensure_loss(h);  // for the device flag
    after_caller(h);
    hip_check(sp::launch_compare_pattern(h->a, row_ptr, col_idx, h->stream));
    int32_t bad = 1;
    hip_check(hipMemcpyAsync(&bad, h->a.bad, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    *same_out = bad ? 0 : 1;
    return GMRES_OK;
  });
}

int spai_destroy(spai_handle hh) {
  if (!hh) return GMRES_OK;
  if (hh->magic != kMagic) return GMRES_EHANDLE;
  delete hh;
  return GMRES_OK;
}

int spai_adam_step(int64_t count, float* theta, uint16_t* params_bf16, const float* grad, float grad_scale,
                   float* m1, float* m2, float lr, float beta1, float beta2, float eps, int32_t t,
                   void* hip_stream) {
  if (count <= 0 || !theta || !params_bf16 || !grad || !m1 || !m2 || t < 1) return GMRES_EINVAL;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f)) return GMRES_EINVAL;
  return guarded([&] {
    hipStream_t st = (hipStream_t)hip_stream;
    hip_check(sp::launch_adam(count, theta, params_bf16, grad, grad_scale, m1, m2, lr, beta1, beta2, eps, t, st));
    hip_check(hipStreamSynchronize(st));
    return GMRES_OK;
  });
}

}  // extern "C"

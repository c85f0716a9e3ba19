// Device blocks of the solver handles, kept for reuse.
//
// A handle allocates some 50 device buffers at create time (the CSR copies,
// the basis, the row-block and segment tables, the partial tables, the
// solution vectors).  A destroyed handle's blocks go back to a per-device
// cache instead of hipFree, so the next handle of the same shape takes them
// without a hipMalloc each (a create is then bound by its own kernels and
// copies).  Blocks are matched by their rounded size; the cache keeps at
// most kCap bytes per device and frees the rest, and a failed hipMalloc
// empties the cache of that device and tries once more.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>

#include "gmres_internal.hpp"

namespace gm {
namespace {

constexpr size_t kCap = size_t(16) << 30;

struct Block {
  int dev;
  size_t bytes;
};

struct Cache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> free;  // device -> size -> block
  std::map<int, size_t> free_bytes;
  std::unordered_map<void*, Block> live;
};

Cache& cache() {
  static Cache* c = new Cache;  // never destroyed: blocks may be released at process exit
  return *c;
}

size_t round_bytes(size_t n) {
  n = n < 256 ? 256 : n;
  const size_t g = n < (size_t(1) << 20) ? 256 : n < (size_t(64) << 20) ? (size_t(128) << 10) : (size_t(2) << 20);
  return (n + g - 1) / g * g;
}

void release_device(Cache& c, int dev) {
  auto it = c.free.find(dev);
  if (it == c.free.end()) return;
  for (auto& kv : it->second) (void)hipFree(kv.second);
  it->second.clear();
  c.free_bytes[dev] = 0;
}

}  // namespace

void* cache_alloc(size_t bytes, size_t* rounded) {
  const size_t nb = round_bytes(bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto& fl = c.free[dev];
  auto it = fl.find(nb);
  void* p = nullptr;
  if (it != fl.end()) {
    p = it->second;
    fl.erase(it);
    c.free_bytes[dev] -= nb;
  } else if (hipMalloc(&p, nb) != hipSuccess) {
    (void)hipGetLastError();
    release_device(c, dev);
    p = nullptr;
    if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  c.live[p] = Block{dev, nb};
  if (rounded) *rounded = nb;
  return p;
}

void cache_free(void* p) {
  if (!p) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  const Block b = it->second;
  c.live.erase(it);
  if (c.free_bytes[b.dev] + b.bytes > kCap) {
    (void)hipFree(p);
    return;
  }
  c.free[b.dev].emplace(b.bytes, p);
  c.free_bytes[b.dev] += b.bytes;
}

size_t cache_release_all() {
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  size_t n = 0;
  for (auto& kv : c.free_bytes) n += kv.second;
  for (auto& kv : c.free) {
    for (auto& blk : kv.second) (void)hipFree(blk.second);
    kv.second.clear();
  }
  for (auto& kv : c.free_bytes) kv.second = 0;
  return n;
}

}  // namespace gm

// hmx_mem.hip -- caching device allocator behind DevBuf.
//
// Blocks are rounded up (512 B below 1 MiB, 2 MiB above) and, when freed, kept in a per-device
// free list keyed by size.  An allocation takes the smallest cached block that is large enough
// and at most twice the request; otherwise it calls hipMalloc, and on failure releases the
// cache and retries once.  A free first waits for the device (the block may still be read by
// queued work), as hipFree does, but keeps the mapping.
#include <map>
#include <mutex>
#include <unordered_map>

#include "hmx_host.h"

namespace hmx {
namespace {

struct Cache {
  std::mutex mu;
  std::unordered_map<void*, std::pair<int, size_t>> live;  // block -> (device, size)
  std::map<int, std::multimap<size_t, void*>> per_dev;
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: blocks live until process exit
  return *c;
}

size_t round_size(size_t b) {
  if (b <= (1u << 20)) return (b + 511) & ~size_t(511);
  const size_t g = size_t(2) << 20;
  return (b + g - 1) / g * g;
}

void release_locked(Cache& c, int dev) {
  auto& fl = c.per_dev[dev];
  for (auto& kv : fl) (void)hipFree(kv.second);
  fl.clear();
}

}  // namespace

void* dev_alloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  int dev = 0;
  HMX_HIP(hipGetDevice(&dev));
  const size_t sz = round_size(bytes);
  Cache& c = cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto& fl = c.per_dev[dev];
    auto it = fl.lower_bound(sz);
    if (it != fl.end() && it->first <= 2 * sz) {
      void* p = it->second;
      c.live[p] = {dev, it->first};
      fl.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> g(c.mu);
      HMX_HIP(hipDeviceSynchronize());
      release_locked(c, dev);
    }
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess) hip_fail(e, "hipMalloc", __FILE__, __LINE__);
  std::lock_guard<std::mutex> g(c.mu);
  c.live[p] = {dev, sz};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  Cache& c = cache();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) {
    (void)hipFree(p);
    return;
  }
  c.per_dev[it->second.first].emplace(it->second.second, p);
  c.live.erase(it);
}

size_t dev_cached_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  size_t b = 0;
  for (const auto& kv : c.per_dev[dev]) b += kv.first;
  return b;
}

void dev_release_cache() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  Cache& c = cache();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(c.mu);
  release_locked(c, dev);
}

}  // namespace hmx

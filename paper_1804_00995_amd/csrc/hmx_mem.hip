// hmx_mem.hip -- caching device allocator behind DevBuf.
//
// Per device, a SegmentCache (hmx_segcache.h) over hipMalloc'd blocks: sizes are rounded (512 B
// below 1 MiB, 2 MiB above); a freed buffer stays mapped and serves a later request of at most
// twice its size; a buffer sized from an estimate can be shrunk to what it used, its tail then
// serving later requests; on hipMalloc failure the entirely free blocks are released and the
// call retried once.  A free or shrink first waits for the device (the memory may still be read
// by queued work), as hipFree does, but keeps the mapping.
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "hmx_host.h"
#include "hmx_segcache.h"

namespace hmx {
namespace {

struct HipBackend {
  void* alloc(size_t sz) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sz);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (e != hipSuccess) hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    return p;
  }
  void* alloc_or_throw(size_t sz, size_t n_blocks, size_t block_bytes, size_t stranded) {
    HMX_HIP(hipDeviceSynchronize());
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      size_t fb = 0, tb = 0;
      (void)hipMemGetInfo(&fb, &tb);
      throw Error(e == hipErrorOutOfMemory ? HMX_ENOMEM : HMX_EDEVICE,
                  "hipMalloc of " + std::to_string(sz) + " bytes failed (" + hipGetErrorString(e) +
                      "); device free " + std::to_string(fb) + " of " + std::to_string(tb) +
                      " bytes; the library holds " + std::to_string(n_blocks) + " blocks of " +
                      std::to_string(block_bytes) + " bytes, " + std::to_string(stranded) +
                      " of them free beside live buffers");
    }
    return p;
  }
  void release(void* p) { (void)hipFree(p); }
};

struct Cache {
  std::mutex mu;
  std::map<int, std::unique_ptr<SegmentCache<HipBackend>>> per_dev;
  std::map<void*, int> owner;  // live buffer -> device
  SegmentCache<HipBackend>& dev(int d) {
    auto& c = per_dev[d];
    if (!c) c = std::make_unique<SegmentCache<HipBackend>>(HipBackend{});
    return *c;
  }
};

Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: blocks live until process exit
  return *c;
}

int current_device() {
  int dev = 0;
  HMX_HIP(hipGetDevice(&dev));
  return dev;
}

}  // namespace

void* dev_alloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  const int dev = current_device();
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  void* p = c.dev(dev).alloc(bytes);
  c.owner[p] = dev;
  return p;
}

void* dev_alloc_block(size_t bytes) {
  if (bytes == 0) return nullptr;
  const int dev = current_device();
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  void* p = c.dev(dev).alloc_block(bytes);
  c.owner[p] = dev;
  return p;
}

size_t dev_shrink(void* p, size_t bytes) {
  if (!p) return 0;
  Cache& c = cache();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.owner.find(p);
  HMX_REQUIRE(it != c.owner.end(), HMX_EINTERNAL, "dev_shrink of a buffer the cache does not hold");
  return c.dev(it->second).shrink(p, bytes);
}

void dev_free(void* p) {
  if (!p) return;
  Cache& c = cache();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.owner.find(p);
  if (it == c.owner.end()) {
    (void)hipFree(p);
    return;
  }
  c.dev(it->second).free(p);
  c.owner.erase(it);
}

size_t dev_cached_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  return c.dev(dev).free_bytes();
}

void dev_release_cache() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  Cache& c = cache();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(c.mu);
  c.dev(dev).release();
}

}  // namespace hmx

// Host check of the device allocator's segment bookkeeping (hmx_segcache.h) on a malloc backend:
// fixed cases (a shrunk buffer's tail serves the next request, frees merge, only entirely free
// blocks are released) and a seeded random sequence of alloc / shrink / free / release, after
// which every step must leave the cache consistent and the live buffers disjoint, with their
// contents intact.  Prints "ok" and exits 0, or names the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../paper_1804_00995_amd/csrc/hmx_segcache.h"

namespace {

struct MallocBackend {
  std::map<void*, size_t>* live;  // blocks handed out -> size
  size_t* budget;                 // bytes the backend may still hand out
  void* alloc(size_t sz) {
    if (sz > *budget) return nullptr;
    void* p = std::malloc(sz);
    *budget -= sz;
    (*live)[p] = sz;
    return p;
  }
  void* alloc_or_throw(size_t sz, size_t, size_t, size_t) {
    void* p = alloc(sz);
    if (!p) throw std::bad_alloc();
    return p;
  }
  void release(void* p) {
    *budget += live->at(p);
    live->erase(p);
    std::free(p);
  }
};

int fails = 0;
void check(bool c, const char* what) {
  if (!c) {
    std::printf("FAILED: %s\n", what);
    ++fails;
  }
}

}  // namespace

int main() {
  using hmx::seg_round;
  const size_t MiB = size_t(1) << 20;
  std::map<void*, size_t> blocks;
  size_t budget = size_t(1) << 40;
  {
    hmx::SegmentCache<MallocBackend> c(MallocBackend{&blocks, &budget});
    // a 64 MiB buffer shrunk to 10 MiB: the tail is free and serves a 40 MiB request
    char* a = (char*)c.alloc(64 * MiB);
    check(c.shrink(a, 10 * MiB + 5) == 12 * MiB, "shrink rounds up to 2 MiB");
    check(c.free_bytes() == 52 * MiB, "tail is free");
    char* b = (char*)c.alloc(40 * MiB);
    check(b == a + 12 * MiB, "tail serves the next request");
    check(c.n_blocks() == 1, "no new block");
    check(c.consistent(), "consistent after reuse");
    // freeing b then a merges the block back into one free segment, which release returns
    c.release();
    check(c.n_blocks() == 1, "a block with live segments is kept");
    c.free(b);
    c.free(a);
    check(c.n_segments() == 1 && c.free_bytes() == 64 * MiB, "frees merge");
    check(c.consistent(), "consistent after merge");
    c.release();
    check(c.n_blocks() == 0 && blocks.empty(), "entirely free block released");
    // a request larger than twice a free segment takes a new block
    char* s = (char*)c.alloc(4 * MiB);
    c.free(s);
    char* t = (char*)c.alloc(10 * MiB);
    check(t != s && c.n_blocks() == 2, "no reuse beyond twice the request");
    // a shrink at or above the size changes nothing; a shrink next to a free segment merges
    check(c.shrink(t, 20 * MiB) == 10 * MiB, "shrink above the size is a no-op");
    char* u = (char*)c.alloc(3 * MiB);  // the 4 MiB segment (within twice 4 MiB)
    check(u == s, "free segment reused");
    c.shrink(u, 1 * MiB);
    check(c.consistent(), "consistent after small shrink");
    c.free(u);
    c.free(t);
    c.release();
    check(c.n_blocks() == 0 && blocks.empty(), "all released");
    // out of backend memory: the free blocks are released and the call retried
    budget = 100 * MiB;
    char* v = (char*)c.alloc(60 * MiB);
    c.free(v);
    char* w = (char*)c.alloc(30 * MiB);  // reuses v's segment (60 <= 2 * 30)
    check(w == v, "reuse within twice");
    c.free(w);
    char* x = (char*)c.alloc(90 * MiB);  // 60 MiB cached + 90 > budget: release, then allocate
    check(x != nullptr && c.n_blocks() == 1, "release and retry on exhaustion");
    c.free(x);
    c.release();
    budget = size_t(1) << 40;
    // a buffer meant to be shrunk takes a block of its own: not a larger cached block (whose
    // tail it would strand), but a whole free block within 1/8 of its size
    char* big = (char*)c.alloc(150 * MiB);
    c.free(big);
    char* pool = (char*)c.alloc_block(80 * MiB);
    check(pool != big && c.n_blocks() == 2, "no larger cached block for a block allocation");
    c.shrink(pool, 50 * MiB);
    check(c.free_bytes() == 150 * MiB + 30 * MiB, "its tail is its own");
    c.free(pool);
    char* again = (char*)c.alloc_block(76 * MiB);
    check(again == pool, "a whole free block within 1/8 is reused");
    c.free(again);
    check(c.consistent(), "consistent after block allocations");
    c.release();
    check(c.n_blocks() == 0, "all released after block allocations");
  }
  // random sequence
  {
    hmx::SegmentCache<MallocBackend> c(MallocBackend{&blocks, &budget});
    std::mt19937_64 rng(12345);
    struct Buf {
      char* p;
      size_t size;  // usable bytes
      unsigned char tag;
    };
    std::vector<Buf> bufs;
    auto fill = [](const Buf& b) { std::memset(b.p, b.tag, b.size); };
    auto intact = [](const Buf& b) {
      for (size_t i = 0; i < b.size; i += 4093)
        if ((unsigned char)b.p[i] != b.tag) return false;
      return (unsigned char)b.p[b.size - 1] == b.tag;
    };
    for (int step = 0; step < 4000; ++step) {
      const int op = (int)(rng() % 10);
      if (op < 4 || bufs.empty()) {
        const size_t req = 1 + rng() % (rng() % 2 ? (3 * MiB) : (256 * size_t(1) << 10));
        char* p = (char*)(rng() % 4 == 0 ? c.alloc_block(req) : c.alloc(req));
        Buf b{p, req, (unsigned char)(1 + rng() % 250)};
        fill(b);
        bufs.push_back(b);
      } else if (op < 6) {
        Buf& b = bufs[rng() % bufs.size()];
        const size_t keep = 1 + rng() % b.size;
        const size_t got = c.shrink(b.p, keep);
        if (got < seg_round(b.size)) b.size = std::min(b.size, got);
      } else if (op < 9) {
        const size_t i = rng() % bufs.size();
        if (!intact(bufs[i])) check(false, "contents intact until free");
        c.free(bufs[i].p);
        bufs.erase(bufs.begin() + i);
      } else {
        c.release();
      }
      if (!c.consistent()) {
        check(false, "consistent after every step");
        break;
      }
      // live buffers disjoint
      std::map<char*, size_t> iv;
      for (const Buf& b : bufs) iv[b.p] = c.live_size(b.p);
      char* end = nullptr;
      for (const auto& kv : iv) {
        if (end && kv.first < end) {
          check(false, "live buffers disjoint");
          break;
        }
        end = kv.first + kv.second;
      }
    }
    for (const Buf& b : bufs) {
      if (!intact(b)) check(false, "contents intact at the end");
      c.free(b.p);
    }
    c.release();
    check(c.n_blocks() == 0 && blocks.empty(), "everything released at the end");
  }
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}

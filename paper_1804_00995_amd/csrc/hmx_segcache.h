// hmx_segcache.h -- bookkeeping of the library's caching device allocator, free of HIP so that
// it can be checked on the host.
//
// A block is one allocation from the backend (hipMalloc on the device).  Each block is cut into
// consecutive segments, live or free, that cover it exactly.  alloc() hands out a whole free
// segment (the smallest one of at least the rounded request and at most twice it) or a new
// block; alloc_block() takes a whole block of about the request's size, for buffers that will be
// shrunk; shrink() keeps the first part of a live segment and frees the rest, so that a buffer
// sized from an estimate can give back what it did not use; free() marks a segment free and
// merges it with free neighbours of the same block; release() returns to the backend the blocks
// that are entirely free.  Segments never cross blocks, so a block goes back to the backend only
// when nothing in it is live.  Not thread-safe: the caller holds a lock.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <stdexcept>

namespace hmx {

// Sizes: multiples of 512 bytes up to 1 MiB, of 2 MiB above (the segment boundaries a shrink
// creates keep that alignment).
inline size_t seg_round(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 511) & ~size_t(511);
  const size_t g = size_t(2) << 20;
  return (b + g - 1) / g * g;
}

template <class Backend>
class SegmentCache {
 public:
  explicit SegmentCache(Backend be) : be_(be) {}

  // A live segment of at least `bytes` (rounded), or nullptr for 0 bytes.  Throws what the
  // backend throws when it cannot allocate (after releasing the free blocks once); the backend
  // is told how many blocks the cache still holds, their bytes and their unreleasable free
  // bytes, for its message.
  void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t sz = seg_round(bytes);
    auto it = free_.lower_bound(sz);
    if (it != free_.end() && it->first <= 2 * sz) {
      char* p = it->second;
      free_.erase(it);
      segs_.at(p).live = true;
      return p;
    }
    char* p = (char*)be_.alloc(sz);
    if (p == nullptr) {
      release();
      size_t nb = 0, bb = 0, sf = 0;
      stats(&nb, &bb, &sf);
      p = (char*)be_.alloc_or_throw(sz, nb, bb, sf);
    }
    blocks_[p] = sz;
    segs_[p] = Seg{p, sz, true};
    return p;
  }

  // A block of its own for a buffer that will be shrunk (a pool sized from an estimate): an
  // entirely free cached block of at least the rounded size and at most 1/8 more, or a new
  // block of exactly that size.  Shrinking it later leaves free only its own unused tail.
  void* alloc_block(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t sz = seg_round(bytes);
    for (auto it = free_.lower_bound(sz); it != free_.end() && it->first <= sz + sz / 8; ++it) {
      char* p = it->second;
      auto b = blocks_.find(p);
      if (b != blocks_.end() && b->second == it->first) {
        free_.erase(it);
        segs_.at(p).live = true;
        return p;
      }
    }
    char* p = (char*)be_.alloc(sz);
    if (p == nullptr) {
      release();
      size_t nb = 0, bb = 0, sf = 0;
      stats(&nb, &bb, &sf);
      p = (char*)be_.alloc_or_throw(sz, nb, bb, sf);
    }
    blocks_[p] = sz;
    segs_[p] = Seg{p, sz, true};
    return p;
  }

  // Keeps the first `bytes` (rounded) of the live segment at p and frees the rest (merged with
  // a free segment that follows it in the same block).  A request at or above the segment's
  // size changes nothing.  Returns the segment's size afterwards.
  size_t shrink(void* vp, size_t bytes) {
    char* p = (char*)vp;
    Seg& s = live_seg(p);
    const size_t keep = seg_round(bytes == 0 ? 1 : bytes);
    if (keep >= s.size) return s.size;
    char* t = p + keep;
    const size_t rest = s.size - keep;
    s.size = keep;
    segs_[t] = Seg{s.block, rest, false};
    add_free(merge_next(t));
    return keep;
  }

  // Frees the live segment at p (merging it with free neighbours of its block).
  void free(void* vp) {
    char* p = (char*)vp;
    Seg& s = live_seg(p);
    s.live = false;
    char* q = merge_next(p);
    // merge with a free predecessor in the same block
    auto it = segs_.find(q);
    if (it != segs_.begin()) {
      auto pv = std::prev(it);
      if (!pv->second.live && pv->second.block == it->second.block &&
          pv->first + pv->second.size == q) {
        drop_free(pv->first, pv->second.size);
        pv->second.size += it->second.size;
        segs_.erase(it);
        q = pv->first;
      }
    }
    add_free(q);
  }

  // Returns every entirely free block to the backend.
  void release() {
    for (auto it = blocks_.begin(); it != blocks_.end();) {
      char* b = it->first;
      const Seg& s = segs_.at(b);
      if (!s.live && s.size == it->second) {
        drop_free(b, s.size);
        segs_.erase(b);
        be_.release(b);
        it = blocks_.erase(it);
      } else {
        ++it;
      }
    }
  }

  // Blocks, their bytes, and the bytes of free segments in blocks that also hold live ones
  // (which release() cannot return).
  void stats(size_t* n_blocks, size_t* block_bytes, size_t* stranded_free) const {
    size_t nb = 0, bb = 0, sf = 0;
    for (const auto& b : blocks_) {
      ++nb;
      bb += b.second;
      const Seg& first = segs_.at(b.first);
      if (!(first.size == b.second && !first.live)) {
        for (auto it = segs_.find(b.first); it != segs_.end() && it->second.block == b.first; ++it)
          if (!it->second.live) sf += it->second.size;
      }
    }
    *n_blocks = nb;
    *block_bytes = bb;
    *stranded_free = sf;
  }

  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& kv : free_) t += kv.first;
    return t;
  }
  size_t live_size(void* p) const {
    auto it = segs_.find((char*)p);
    return it != segs_.end() && it->second.live ? it->second.size : 0;
  }
  bool owns(void* p) const {
    auto it = segs_.find((char*)p);
    return it != segs_.end() && it->second.live;
  }
  size_t n_blocks() const { return blocks_.size(); }
  size_t n_segments() const { return segs_.size(); }

  // Every block is covered by consecutive segments; no two free neighbours in one block; the
  // free index lists exactly the free segments.  Returns false on the first violation.
  bool consistent() const {
    size_t nfree = 0, nseg = 0;
    for (const auto& b : blocks_) {
      char* p = b.first;
      bool prev_free = false;
      while (p < b.first + b.second) {
        auto it = segs_.find(p);
        if (it == segs_.end() || it->second.block != b.first || it->second.size == 0) return false;
        if (!it->second.live) {
          if (prev_free) return false;
          ++nfree;
          bool listed = false;
          auto r = free_.equal_range(it->second.size);
          for (auto f = r.first; f != r.second; ++f) listed = listed || f->second == p;
          if (!listed) return false;
        }
        prev_free = !it->second.live;
        p += it->second.size;
        ++nseg;
      }
      if (p != b.first + b.second) return false;
    }
    return nfree == free_.size() && nseg == segs_.size();
  }

 private:
  struct Seg {
    char* block;
    size_t size;
    bool live;
  };

  Seg& live_seg(char* p) {
    auto it = segs_.find(p);
    if (it == segs_.end() || !it->second.live)
      throw std::logic_error("segment cache: pointer is not a live segment");
    return it->second;
  }
  void add_free(char* p) { free_.emplace(segs_.at(p).size, p); }
  void drop_free(char* p, size_t size) {
    auto r = free_.equal_range(size);
    for (auto f = r.first; f != r.second; ++f)
      if (f->second == p) {
        free_.erase(f);
        return;
      }
  }
  // Merges the free segment at p with a free successor in the same block; returns p.
  char* merge_next(char* p) {
    auto it = segs_.find(p);
    auto nx = std::next(it);
    if (nx != segs_.end() && !nx->second.live && nx->second.block == it->second.block &&
        p + it->second.size == nx->first) {
      drop_free(nx->first, nx->second.size);
      it->second.size += nx->second.size;
      segs_.erase(nx);
    }
    return p;
  }

  Backend be_;
  std::map<char*, size_t> blocks_;      // block -> size
  std::map<char*, Seg> segs_;           // segment start -> segment
  std::multimap<size_t, char*> free_;   // free segments by size
};

}  // namespace hmx

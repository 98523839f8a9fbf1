// k_sort.hip -- radix sort of (64-bit key, 32-bit value) pairs, used to put the near and far
// block lists in their defined order.  The keys are unique, so the result is fully determined.
//
// Least-significant-digit radix sort, 8-bit digits, ceil(end_bit / 8) passes.  Each pass:
//   sort_hist:    workgroup b counts the digits of its chunk of SORT_CHUNK items into
//                 hist[d * G + b] (G workgroups);
//   scan:         exclusive scan of hist in that digit-major order gives every (digit, chunk)
//                 its first output position;
//   sort_scatter: workgroup b walks its chunk in tiles of WG items, in order; an item's position
//                 is its (digit, chunk) base, plus the items of its digit in earlier wavefronts of
//                 the tile, plus those in earlier lanes of its wavefront (eight ballots give the
//                 lanes with the same digit).  Items keep their relative order within a digit,
//                 so each pass is stable and the passes compose into a full sort.
#include <algorithm>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

namespace {

constexpr int SORT_TILES = 8;                  // tiles of WG items per chunk
constexpr int SORT_CHUNK = WG * SORT_TILES;   // items per workgroup
constexpr int RADIX = 256;

__global__ void __launch_bounds__(WG) sort_hist_kernel(const uint64_t* __restrict__ key,
                                                       int64_t n, int shift,
                                                       int64_t* __restrict__ hist) {
  __shared__ int cnt[RADIX];
  const int b = blockIdx.x, G = gridDim.x;
  cnt[threadIdx.x] = 0;  // WG == RADIX
  __syncthreads();
  const int64_t i0 = (int64_t)b * SORT_CHUNK;
  for (int t = 0; t < SORT_TILES; ++t) {
    const int64_t i = i0 + t * WG + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((key[i] >> shift) & (RADIX - 1))], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * G + b] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(WG) sort_scatter_kernel(
    const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    const int64_t* __restrict__ offs, uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ int64_t base[RADIX];
  __shared__ int wcnt[NWAVE][RADIX];
  const int b = blockIdx.x, G = gridDim.x;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * G + b];
  const int64_t i0 = (int64_t)b * SORT_CHUNK;
  const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
  for (int t = 0; t < SORT_TILES; ++t) {
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) wcnt[q][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = i0 + t * WG + threadIdx.x;
    const bool valid = i < n;
    const uint64_t k = valid ? kin[i] : 0ull;
    const int d = (int)((k >> shift) & (RADIX - 1));
    // lanes of this wavefront holding an item with the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t m = __ballot((d >> bit) & 1);
      same &= ((d >> bit) & 1) ? m : ~m;
    }
    const int before = __popcll(same & below);
    if (valid && before == 0) wcnt[w][d] = __popcll(same);  // the digit's first lane
    __syncthreads();
    if (valid) {
      int64_t pos = base[d] + before;
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      kout[pos] = k;
      vout[pos] = vin[i];
    }
    __syncthreads();
    {
      const int dd = threadIdx.x;  // one digit per thread: advance its base past this tile
      int64_t add = 0;
#pragma unroll
      for (int q = 0; q < NWAVE; ++q) add += wcnt[q][dd];
      base[dd] += add;
    }
  }
}

}  // namespace

void radix_sort_u64_pairs(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout,
                          int64_t n, int end_bit, DevBuf<unsigned char>& tmp, hipStream_t s) {
  static_assert(WG == RADIX, "one digit per thread");
  if (n <= 0) return;
  const int passes = std::max(1, (end_bit + 7) / 8);
  const int64_t G = (n + SORT_CHUNK - 1) / SORT_CHUNK;
  HMX_REQUIRE(G <= (int64_t)1 << 30, HMX_EUNSUPPORTED, "too many items to sort");
  // scratch: two ping-pong key and value buffers, the histogram and its scan
  const size_t kb = (size_t)n * 8, vb = (size_t)n * 4, hb = (size_t)RADIX * G * 8;
  const size_t a8 = (kb + 255) & ~size_t(255);
  const size_t av = (vb + 255) & ~size_t(255), ah = (hb + 255) & ~size_t(255);
  const size_t aw = (size_t)scan_work_len((int64_t)RADIX * G) * 8;
  tmp.alloc(2 * a8 + 2 * av + ah + ah + 8 + aw + 8);
  unsigned char* p = tmp.p;
  uint64_t* kbuf[2] = {(uint64_t*)p, (uint64_t*)(p + a8)};
  int32_t* vbuf[2] = {(int32_t*)(p + 2 * a8), (int32_t*)(p + 2 * a8 + av)};
  int64_t* hist = (int64_t*)(p + 2 * a8 + 2 * av);
  int64_t* offs = (int64_t*)(p + 2 * a8 + 2 * av + ah);  // RADIX G + 1 entries
  int64_t* work = (int64_t*)(p + 2 * a8 + 2 * av + 2 * ah + 8);  // the scan's block sums
  for (int pass = 0; pass < passes; ++pass) {
    const uint64_t* ki = pass == 0 ? kin : kbuf[(pass - 1) & 1];
    const int32_t* vi = pass == 0 ? vin : vbuf[(pass - 1) & 1];
    uint64_t* ko = pass == passes - 1 ? kout : kbuf[pass & 1];
    int32_t* vo = pass == passes - 1 ? vout : vbuf[pass & 1];
    const int shift = 8 * pass;
    hipLaunchKernelGGL(sort_hist_kernel, dim3((unsigned)G), dim3(WG), 0, s, ki, n, shift, hist);
    HMX_LAUNCHED();
    scan_excl_i64_work(hist, offs, RADIX * G, work, s);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)G), dim3(WG), 0, s, ki, vi, n, shift,
                       offs, ko, vo);
    HMX_LAUNCHED();
  }
}

}  // namespace hmx

// k_blocks.hip -- block tree (admissibility), sorting of the block lists and the per-leaf /
// per-node index structures used by the product.
//
// Definition (the paper leaves it unstated): diam(t) is the length of the box diagonal and
// dist(t, s) the Euclidean distance between the two boxes (0 when they overlap).  Starting from
// (root, root), a pair is far (admissible) when min(diam_t^2, diam_s^2) <= eta^2 dist^2; otherwise
// it is near when both nodes are leaves; otherwise the non-leaf side(s) are split into their
// children (2 or 4 pairs).  The traversal is level synchronous: one thread per pair of the
// current frontier, every level queued by the host before any size is read back.  Compiled without floating-point contraction so that the squared sizes are
// evaluated exactly as written.
#include <algorithm>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

__device__ __forceinline__ double diam2(const double* bx) {
  double ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
  return ex * ex + ey * ey + ez * ez;
}
__device__ __forceinline__ double dist2(const double* a, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double g = 0.0;
    if (b[d] - a[3 + d] > g) g = b[d] - a[3 + d];
    if (a[d] - b[3 + d] > g) g = a[d] - b[3 + d];
    s = s + g * g;
  }
  return s;
}

// Row shares: only pairs whose row node meets the point range [rb, re) (cluster positions) are
// followed, and a block is emitted only when its row node lies inside the range; a block that
// would straddle the range sets bit 1 of *err (the caller picks the range as a node below every
// emitted block).  rb = 0, re = M keeps everything.
//
// One level of the recursion.  Its frontier size is read from the device (*nfront_p, of which
// at most front_cap pairs are in `front`) and the pairs are taken in a grid-stride loop, so the
// host queues every level without reading a size back.  An output past its buffer's capacity
// is dropped and sets bit 2 of *err; the counters still count it, so the host learns the size
// the level needed, and every later level returns at once (its frontier would hold entries
// that were never written).  The host then runs the recursion again with larger buffers.
__global__ void __launch_bounds__(WG) block_level_kernel(
    const int2* __restrict__ front, const int* __restrict__ nfront_p, int64_t front_cap,
    const double* __restrict__ box, const int32_t* __restrict__ child0,
    const int32_t* __restrict__ child1, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, int rb, int re, double eta2, int max_mn,
    int2* __restrict__ next, int64_t next_cap, int* next_cnt, int2* __restrict__ nearL,
    int64_t near_cap, int* near_cnt, int2* __restrict__ farL, int64_t far_cap, int* far_cnt,
    int* err) {
  // after a dropped output the frontier is incomplete (and holds unwritten entries): the levels
  // that follow do nothing, and the host runs the recursion again with larger buffers
  if (*err & 2) return;
  const int64_t nfront = min((int64_t)*nfront_p, front_cap);
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < nfront; i += stride) {
    const int2 ts = front[i];
    const int t = ts.x, s = ts.y;
    const int tb = nbegin[t], te = nend[t];
    if (te <= rb || tb >= re) continue;  // rows outside the share
    const bool inside = tb >= rb && te <= re;
    const double* bt = box + 6 * (int64_t)t;
    const double* bs = box + 6 * (int64_t)s;
    const double dt = diam2(bt), ds = diam2(bs);
    const double dmin = dt < ds ? dt : ds;
    const int t0 = child0[t], s0 = child0[s];
    const bool lt = t0 < 0, ls = s0 < 0;
    // an admissible pair is far unless it exceeds max_mn points (then its children are taken,
    // down to leaf pairs, which are far whatever their size)
    const bool small = max_mn <= 0 || (te - tb) + (nend[s] - nbegin[s]) <= max_mn || (lt && ls);
    if (small && dmin <= eta2 * dist2(bt, bs)) {
      if (!inside) {
        atomicOr(err, 1);
      } else {
        const int q = atomicAdd(far_cnt, 1);
        if (q < far_cap) farL[q] = ts;
        else atomicOr(err, 2);
      }
      continue;
    }
    if (!small && lt && ls) continue;  // unreachable: leaf pairs are small
    if (lt && ls) {
      if (!inside) {
        atomicOr(err, 1);
      } else {
        const int q = atomicAdd(near_cnt, 1);
        if (q < near_cap) nearL[q] = ts;
        else atomicOr(err, 2);
      }
      continue;
    }
    // the children of the non-leaf side(s): 2 or 4 pairs
    int2 c[4];
    int nc;
    if (lt) {
      c[0] = make_int2(t, s0);
      c[1] = make_int2(t, child1[s]);
      nc = 2;
    } else if (ls) {
      c[0] = make_int2(t0, s);
      c[1] = make_int2(child1[t], s);
      nc = 2;
    } else {
      const int t1 = child1[t], s1 = child1[s];
      c[0] = make_int2(t0, s0);
      c[1] = make_int2(t0, s1);
      c[2] = make_int2(t1, s0);
      c[3] = make_int2(t1, s1);
      nc = 4;
    }
    const int q = atomicAdd(next_cnt, nc);
    if (q + nc <= next_cap) {
      for (int j = 0; j < nc; ++j) next[q + j] = c[j];
    } else {
      atomicOr(err, 2);
    }
  }
}

void launch_block_level(const int2* front, const int* nfront, int64_t front_cap,
                        const double* box, const int32_t* child0, const int32_t* child1,
                        const int32_t* nbegin, const int32_t* nend, int rb, int re, double eta2,
                        int max_mn, int2* next, int64_t next_cap, int* next_cnt, int2* nearL,
                        int64_t near_cap, int* near_cnt, int2* farL, int64_t far_cap,
                        int* far_cnt, int* err, hipStream_t s) {
  // a fixed grid: the frontier size is known only on the device
  const int64_t want = (front_cap + WG - 1) / WG;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 512));
  hipLaunchKernelGGL(block_level_kernel, dim3(grid), dim3(WG), 0, s, front, nfront, front_cap,
                     box, child0, child1, nbegin, nend, rb, re, eta2, max_mn, next, next_cap,
                     next_cnt, nearL, near_cap, near_cnt, farL, far_cap, far_cnt, err);
  HMX_LAUNCHED();
}

// Rank of every cluster-tree node in the order of (begin, end), for short sort keys.  The nodes
// that start at one position p form a chain of left children at consecutive levels (a node
// that is not a leaf starts where its left child starts), and the deeper one ends first, so
//   rank = start[p] + (deepest level starting at p - level),
// with start the exclusive scan of the number of nodes starting at each position.
__global__ void node_begin_count_kernel(const int32_t* __restrict__ nbegin,
                                        const int32_t* __restrict__ level, int n_nodes,
                                        int64_t* __restrict__ cnt, int32_t* __restrict__ deep) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n_nodes) return;
  atomicAdd((unsigned long long*)&cnt[nbegin[i]], 1ull);
  atomicMax(&deep[nbegin[i]], level[i]);
}
__global__ void node_rank_kernel(const int32_t* __restrict__ nbegin,
                                 const int32_t* __restrict__ level, int n_nodes,
                                 const int64_t* __restrict__ start,
                                 const int32_t* __restrict__ deep, int32_t* __restrict__ rank) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n_nodes) return;
  const int p = nbegin[i];
  rank[i] = (int32_t)(start[p] + (deep[p] - level[i]));
}
void launch_node_rank(const int32_t* nbegin, const int32_t* level, int n_nodes, int64_t M,
                      int64_t* cnt, int64_t* start, int32_t* deep, int32_t* rank, hipStream_t s) {
  fill_i64(cnt, 0, M, s);
  fill_i32(deep, -1, M, s);
  const unsigned g = (unsigned)((n_nodes + WG - 1) / WG);
  hipLaunchKernelGGL(node_begin_count_kernel, dim3(g), dim3(WG), 0, s, nbegin, level, n_nodes, cnt,
                     deep);
  HMX_LAUNCHED();
  scan_excl_i64(cnt, start, M, s);
  hipLaunchKernelGGL(node_rank_kernel, dim3(g), dim3(WG), 0, s, nbegin, level, n_nodes, start, deep,
                     rank);
  HMX_LAUNCHED();
}

// Keys of a block list from the node ranks: (list << 2 bits) | rank_t * n_nodes + rank_s, whose
// order is the lexicographic order of (list, t.begin, t.end, s.begin, s.end); val = the pair's
// index in the concatenated lists (offset + i).
__global__ void pair_rank_keys_kernel(const int2* __restrict__ pairs, int64_t n,
                                      const int32_t* __restrict__ rank, int64_t n_nodes,
                                      uint64_t list_bit, int64_t offset,
                                      uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const int2 p = pairs[i];
  key[offset + i] = list_bit | ((uint64_t)rank[p.x] * (uint64_t)n_nodes + (uint64_t)rank[p.y]);
  val[offset + i] = (int32_t)(offset + i);
}
void launch_pair_rank_keys(const int2* pairs, int64_t n, const int32_t* rank, int64_t n_nodes,
                           uint64_t list_bit, int64_t offset, uint64_t* key, int32_t* val,
                           hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(pair_rank_keys_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s,
                     pairs, n, rank, n_nodes, list_bit, offset, key, val);
  HMX_LAUNCHED();
}

// out[i] = the pair at index idx[i] of the concatenated lists (a, na entries, then b)
__global__ void pair_gather2_kernel(const int2* __restrict__ a, int64_t na,
                                    const int2* __restrict__ b, const int32_t* __restrict__ idx,
                                    int64_t n, int2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const int64_t j = idx[i];
  out[i] = j < na ? a[j] : b[j - na];
}
void launch_pair_gather2(const int2* a, int64_t na, const int2* b, const int32_t* idx, int64_t n,
                         int2* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(pair_gather2_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, a,
                     na, b, idx, n, out);
  HMX_LAUNCHED();
}

// Near blocks (sorted): entry counts m*n for the pool offsets, and blocks per row leaf.
__global__ void near_prep_kernel(const int2* __restrict__ nearL, int64_t n,
                                 const int32_t* __restrict__ nbegin, const int32_t* __restrict__ nend,
                                 const int32_t* __restrict__ leaf_of_node, int64_t* __restrict__ sizes,
                                 int64_t* __restrict__ leaf_cnt) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  int2 p = nearL[i];
  int64_t m = nend[p.x] - nbegin[p.x], c = nend[p.y] - nbegin[p.y];
  sizes[i] = m * c;
  atomicAdd((unsigned long long*)&leaf_cnt[leaf_of_node[p.x]], 1ull);
}
void launch_near_prep(const int2* nearL, int64_t n, const int32_t* nbegin, const int32_t* nend,
                      const int32_t* leaf_of_node, int64_t* sizes, int64_t* leaf_cnt, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(near_prep_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, nearL,
                     n, nbegin, nend, leaf_of_node, sizes, leaf_cnt);
  HMX_LAUNCHED();
}

// Far blocks (sorted): ranges, far-block count per row node and the first block of each node
// (blocks of one row node are contiguous in the sorted list).
__global__ void far_prep_kernel(const int2* __restrict__ farL, int64_t n,
                                const int32_t* __restrict__ nbegin, const int32_t* __restrict__ nend,
                                int32_t* __restrict__ far_tb, int32_t* __restrict__ far_m,
                                int32_t* __restrict__ far_sb, int32_t* __restrict__ far_n,
                                int64_t* __restrict__ node_cnt, int32_t* __restrict__ node_first) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  int2 p = farL[i];
  far_tb[i] = nbegin[p.x];
  far_m[i] = nend[p.x] - nbegin[p.x];
  far_sb[i] = nbegin[p.y];
  far_n[i] = nend[p.y] - nbegin[p.y];
  atomicAdd((unsigned long long*)&node_cnt[p.x], 1ull);
  if (i == 0 || farL[i - 1].x != p.x) node_first[p.x] = (int32_t)i;
}
void launch_far_prep(const int2* farL, int64_t n, const int32_t* nbegin, const int32_t* nend,
                     int32_t* far_tb, int32_t* far_m, int32_t* far_sb, int32_t* far_n,
                     int64_t* node_cnt, int32_t* node_first, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(far_prep_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, farL, n,
                     nbegin, nend, far_tb, far_m, far_sb, far_n, node_cnt, node_first);
  HMX_LAUNCHED();
}

// Node ranges of a list of (t, s) pairs.
__global__ void pair_ranges_kernel(const int2* __restrict__ pairs, int64_t n,
                                   const int32_t* __restrict__ nbegin, const int32_t* __restrict__ nend,
                                   int32_t* __restrict__ tb, int32_t* __restrict__ m,
                                   int32_t* __restrict__ sb, int32_t* __restrict__ nn) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  int2 p = pairs[i];
  tb[i] = nbegin[p.x];
  m[i] = nend[p.x] - nbegin[p.x];
  sb[i] = nbegin[p.y];
  nn[i] = nend[p.y] - nbegin[p.y];
}
void launch_pair_ranges(const int2* pairs, int64_t n, const int32_t* nbegin, const int32_t* nend,
                        int32_t* tb, int32_t* m, int32_t* sb, int32_t* nn, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(pair_ranges_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, pairs,
                     n, nbegin, nend, tb, m, sb, nn);
  HMX_LAUNCHED();
}

// For each leaf: the far blocks whose row node contains it, i.e. the far blocks of the leaf and
// of each of its ancestors, listed from the leaf upwards (a fixed, deterministic order).
__global__ void leaf_far_count_kernel(int n_leaves, const int32_t* __restrict__ leaves,
                                      const int32_t* __restrict__ parent,
                                      const int64_t* __restrict__ node_cnt, int64_t* __restrict__ leaf_cnt) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n_leaves) return;
  int64_t c = 0;
  for (int a = leaves[i]; a >= 0; a = parent[a]) c += node_cnt[a];
  leaf_cnt[i] = c;
}
void launch_leaf_far_count(int n_leaves, const int32_t* leaves, const int32_t* parent,
                           const int64_t* node_cnt, int64_t* leaf_cnt, hipStream_t s) {
  hipLaunchKernelGGL(leaf_far_count_kernel, dim3((n_leaves + WG - 1) / WG), dim3(WG), 0, s,
                     n_leaves, leaves, parent, node_cnt, leaf_cnt);
  HMX_LAUNCHED();
}
__global__ void leaf_far_fill_kernel(int n_leaves, const int32_t* __restrict__ leaves,
                                     const int32_t* __restrict__ parent,
                                     const int64_t* __restrict__ node_cnt,
                                     const int32_t* __restrict__ node_first,
                                     const int64_t* __restrict__ leaf_ptr, int32_t* __restrict__ list) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n_leaves) return;
  int64_t q = leaf_ptr[i];
  for (int a = leaves[i]; a >= 0; a = parent[a]) {
    int64_t c = node_cnt[a];
    for (int64_t j = 0; j < c; ++j) list[q++] = node_first[a] + (int32_t)j;
  }
}
void launch_leaf_far_fill(int n_leaves, const int32_t* leaves, const int32_t* parent,
                          const int64_t* node_cnt, const int32_t* node_first,
                          const int64_t* leaf_ptr, int32_t* list, hipStream_t s) {
  hipLaunchKernelGGL(leaf_far_fill_kernel, dim3((n_leaves + WG - 1) / WG), dim3(WG), 0, s,
                     n_leaves, leaves, parent, node_cnt, node_first, leaf_ptr, list);
  HMX_LAUNCHED();
}

}  // namespace hmx

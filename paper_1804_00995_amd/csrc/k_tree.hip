// k_tree.hip -- geometric cluster tree, built level by level on the device.
//
// Definition (the paper leaves the clustering unstated): a node holds a contiguous range
// [begin, end) of the cluster ordering; its box is the tight axis-aligned box of its points.
// A node with more than L points is split along its longest box side (ties x < y < z) at the
// midpoint 0.5 * (lo + hi): points with coordinate < mid form the first child, the rest the
// second, each keeping its relative order (stable partition).  A node whose box has zero
// extent, or whose split would leave one side empty, is a leaf.
//
// One workgroup owns one node of the current level: it reduces the box, decides the split and
// performs the stable partition of its range (chunked workgroup prefix sums), reading the
// current buffers and writing the next ones; levels of few large nodes spread each node over
// many workgroups instead (below).  Nodes are numbered breadth first.
// Compiled without floating-point contraction so that box sizes and midpoints are evaluated
// exactly as written.
#include <float.h>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

__device__ __forceinline__ double wave_minf(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ __forceinline__ double wave_maxf(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

__global__ void __launch_bounds__(WG) tree_level_kernel(
    int first, const int32_t* __restrict__ nbegin, const int32_t* __restrict__ nend, int leaf,
    const double* __restrict__ cx, const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ cw, const int32_t* __restrict__ cperm, double* __restrict__ nx,
    double* __restrict__ ny, double* __restrict__ nz, double* __restrict__ nw,
    int32_t* __restrict__ nperm, double* __restrict__ box, int32_t* __restrict__ nleft) {
  __shared__ double sred[6 * NWAVE];
  __shared__ int sint[NWAVE];
  const int node = first + blockIdx.x;
  const int b = nbegin[node], e = nend[node];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;

  // tight box
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int p = b + tid; p < e; p += WG) {
    double c[3] = {cx[p], cy[p], cz[p]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], c[d]);
      hi[d] = fmax(hi[d], c[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_minf(lo[d]);
    hi[d] = wave_maxf(hi[d]);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sred[d * NWAVE + w] = lo[d];
      sred[(3 + d) * NWAVE + w] = hi[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double l = sred[d * NWAVE], h = sred[(3 + d) * NWAVE];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) {
      l = fmin(l, sred[d * NWAVE + q]);
      h = fmax(h, sred[(3 + d) * NWAVE + q]);
    }
    lo[d] = l;
    hi[d] = h;
  }
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      box[6 * (int64_t)node + d] = lo[d];
      box[6 * (int64_t)node + 3 + d] = hi[d];
    }
  }

  // split decision
  int axis = 0;
  double ext = hi[0] - lo[0];
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    double x = hi[d] - lo[d];
    if (x > ext) {
      ext = x;
      axis = d;
    }
  }
  const int n = e - b;
  bool is_leaf = (n <= leaf) || !(ext > 0.0);
  const double mid = 0.5 * (lo[axis] + hi[axis]);
  const double* ca = axis == 0 ? cx : (axis == 1 ? cy : cz);
  int nl = 0;
  if (!is_leaf) {
    int cnt = 0;
    for (int p = b + tid; p < e; p += WG) cnt += ca[p] < mid ? 1 : 0;
    int tot;
    block_excl_scan(cnt, sint, &tot);
    nl = tot;
    if (nl == 0 || nl == n) is_leaf = true;
  }
  if (is_leaf) {
    for (int p = b + tid; p < e; p += WG) {
      nx[p] = cx[p];
      ny[p] = cy[p];
      nz[p] = cz[p];
      nw[p] = cw[p];
      nperm[p] = cperm[p];
    }
    if (tid == 0) nleft[node] = -1;
    return;
  }
  // stable partition, one chunk of WG points at a time
  int left_before = 0;
  for (int c = b; c < e; c += WG) {
    int p = c + tid;
    bool valid = p < e;
    bool isl = valid && ca[p] < mid;
    int tot;
    int pre = block_excl_scan(isl ? 1 : 0, sint, &tot);
    if (valid) {
      int q = isl ? b + left_before + pre : b + nl + (p - b - (left_before + pre));
      nx[q] = cx[p];
      ny[q] = cy[p];
      nz[q] = cz[p];
      nw[q] = cw[p];
      nperm[q] = cperm[p];
    }
    left_before += tot;
  }
  if (tid == 0) nleft[node] = nl;
}

void launch_tree_level(int first, int count, const int32_t* nbegin, const int32_t* nend, int leaf,
                       const double* cx, const double* cy, const double* cz, const double* cw,
                       const int32_t* cperm, double* nx, double* ny, double* nz, double* nw,
                       int32_t* nperm, double* box, int32_t* nleft, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(tree_level_kernel, dim3(count), dim3(WG), 0, s, first, nbegin, nend, leaf, cx,
                     cy, cz, cw, cperm, nx, ny, nz, nw, nperm, box, nleft);
  HMX_LAUNCHED();
}

// ------------------------------------------------------------------ multi-workgroup level
// The same level step for levels of few, large nodes: each node's range is cut into chunks of
// TREE_CHUNK points handled by separate workgroups, and the per-node steps (box, split decision,
// left count) combine the chunks' partial results.  Every result equals that of the
// one-workgroup kernel above (min / max and counts do not depend on the order).
constexpr int TREE_CHUNK = 2048;

// Largest i with choff[i] <= ch: the node (index within the level) owning chunk ch.
__device__ __forceinline__ int chunk_node(const int32_t* __restrict__ choff, int count, int ch) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (choff[mid] <= ch) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Chunk offsets of the level's nodes: choff[i] = sum_{q < i} ceil(n_q / TREE_CHUNK).
__global__ void __launch_bounds__(WG) tree_chunk_offsets_kernel(
    int first, int count, const int32_t* __restrict__ nbegin, const int32_t* __restrict__ nend,
    int32_t* __restrict__ choff) {
  __shared__ int s[NWAVE];
  int run = 0;
  for (int c = 0; c < count; c += WG) {
    const int i = c + threadIdx.x;
    int nc = 0;
    if (i < count) nc = (nend[first + i] - nbegin[first + i] + TREE_CHUNK - 1) / TREE_CHUNK;
    int tot;
    const int pre = block_excl_scan(nc, s, &tot);
    if (i < count) choff[i] = run + pre;
    run += tot;
  }
  if (threadIdx.x == 0) choff[count] = run;
}

// Partial box of each chunk.
__global__ void __launch_bounds__(WG) tree_chunk_box_kernel(
    int first, int count, const int32_t* __restrict__ choff, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz, double* __restrict__ pbox) {
  __shared__ double sred[6 * NWAVE];
  const int ch = blockIdx.x;
  if (ch >= choff[count]) return;
  const int i = chunk_node(choff, count, ch), node = first + i;
  const int b = nbegin[node] + (ch - choff[i]) * TREE_CHUNK;
  const int e = min(b + TREE_CHUNK, nend[node]);
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int p = b + tid; p < e; p += WG) {
    const double c[3] = {cx[p], cy[p], cz[p]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], c[d]);
      hi[d] = fmax(hi[d], c[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_minf(lo[d]);
    hi[d] = wave_maxf(hi[d]);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sred[d * NWAVE + w] = lo[d];
      sred[(3 + d) * NWAVE + w] = hi[d];
    }
  }
  __syncthreads();
  if (tid < 3) {
    double l = sred[tid * NWAVE], h = sred[(3 + tid) * NWAVE];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) {
      l = fmin(l, sred[tid * NWAVE + q]);
      h = fmax(h, sred[(3 + tid) * NWAVE + q]);
    }
    pbox[6 * (int64_t)ch + tid] = l;
    pbox[6 * (int64_t)ch + 3 + tid] = h;
  }
}

// Per node: box from the chunk boxes, split axis and midpoint (axis -1: a leaf by size or extent).
__global__ void __launch_bounds__(WG) tree_node_split_kernel(
    int first, int count, const int32_t* __restrict__ choff, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, int leaf, const double* __restrict__ pbox,
    double* __restrict__ box, int32_t* __restrict__ saxis, double* __restrict__ smid) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= count) return;
  const int node = first + i;
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int ch = choff[i]; ch < choff[i + 1]; ++ch) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], pbox[6 * (int64_t)ch + d]);
      hi[d] = fmax(hi[d], pbox[6 * (int64_t)ch + 3 + d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    box[6 * (int64_t)node + d] = lo[d];
    box[6 * (int64_t)node + 3 + d] = hi[d];
  }
  int axis = 0;
  double ext = hi[0] - lo[0];
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    const double x = hi[d] - lo[d];
    if (x > ext) {
      ext = x;
      axis = d;
    }
  }
  const bool is_leaf = (nend[node] - nbegin[node] <= leaf) || !(ext > 0.0);
  saxis[i] = is_leaf ? -1 : axis;
  smid[i] = 0.5 * (lo[axis] + hi[axis]);
}

// Points left of the midpoint in each chunk of a splitting node.
__global__ void __launch_bounds__(WG) tree_chunk_count_kernel(
    int first, int count, const int32_t* __restrict__ choff, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const int32_t* __restrict__ saxis, const double* __restrict__ smid,
    int32_t* __restrict__ ccnt) {
  __shared__ int s[NWAVE];
  const int ch = blockIdx.x;
  if (ch >= choff[count]) return;
  const int i = chunk_node(choff, count, ch), node = first + i;
  const int axis = saxis[i];
  if (axis < 0) return;
  const int b = nbegin[node] + (ch - choff[i]) * TREE_CHUNK;
  const int e = min(b + TREE_CHUNK, nend[node]);
  const double* ca = axis == 0 ? cx : (axis == 1 ? cy : cz);
  const double mid = smid[i];
  int cnt = 0;
  for (int p = b + threadIdx.x; p < e; p += WG) cnt += ca[p] < mid ? 1 : 0;
  int tot;
  block_excl_scan(cnt, s, &tot);
  if (threadIdx.x == 0) ccnt[ch] = tot;
}

// Per node: left points before each chunk (exclusive scan over the node's chunks), the left
// count, and the leaf decision for a split that leaves one side empty.
__global__ void __launch_bounds__(WG) tree_node_left_kernel(
    int first, int count, const int32_t* __restrict__ choff, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, int32_t* __restrict__ saxis,
    const int32_t* __restrict__ ccnt, int32_t* __restrict__ cleft, int32_t* __restrict__ nleft) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= count) return;
  const int node = first + i;
  if (saxis[i] < 0) {
    nleft[node] = -1;
    return;
  }
  int run = 0;
  for (int ch = choff[i]; ch < choff[i + 1]; ++ch) {
    cleft[ch] = run;
    run += ccnt[ch];
  }
  const int n = nend[node] - nbegin[node];
  if (run == 0 || run == n) {
    saxis[i] = -1;
    nleft[node] = -1;
  } else {
    nleft[node] = run;
  }
}

// Stable partition of each chunk into the next buffers (a leaf's chunk is copied in place).
__global__ void __launch_bounds__(WG) tree_chunk_scatter_kernel(
    int first, int count, const int32_t* __restrict__ choff, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const int32_t* __restrict__ saxis,
    const double* __restrict__ smid, const int32_t* __restrict__ cleft,
    const int32_t* __restrict__ nleft, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz, const double* __restrict__ cw,
    const int32_t* __restrict__ cperm, double* __restrict__ nx, double* __restrict__ ny,
    double* __restrict__ nz, double* __restrict__ nw, int32_t* __restrict__ nperm) {
  __shared__ int s[NWAVE];
  const int ch = blockIdx.x;
  if (ch >= choff[count]) return;
  const int i = chunk_node(choff, count, ch), node = first + i;
  const int nb = nbegin[node];
  const int b = nb + (ch - choff[i]) * TREE_CHUNK;
  const int e = min(b + TREE_CHUNK, nend[node]);
  const int axis = saxis[i];
  if (axis < 0) {
    for (int p = b + threadIdx.x; p < e; p += WG) {
      nx[p] = cx[p];
      ny[p] = cy[p];
      nz[p] = cz[p];
      nw[p] = cw[p];
      nperm[p] = cperm[p];
    }
    return;
  }
  const double* ca = axis == 0 ? cx : (axis == 1 ? cy : cz);
  const double mid = smid[i];
  const int nl = nleft[node];
  int left_before = cleft[ch];                   // left points of the node before position c
  for (int c = b; c < e; c += WG) {
    const int p = c + threadIdx.x;
    const bool valid = p < e;
    const bool isl = valid && ca[p] < mid;
    int tot;
    const int pre = block_excl_scan(isl ? 1 : 0, s, &tot);
    if (valid) {
      const int q = isl ? nb + left_before + pre : nb + nl + (p - nb - (left_before + pre));
      nx[q] = cx[p];
      ny[q] = cy[p];
      nz[q] = cz[p];
      nw[q] = cw[p];
      nperm[q] = cperm[p];
    }
    left_before += tot;
  }
}

void launch_tree_level_chunked(int first, int count, int max_chunks, const int32_t* nbegin,
                               const int32_t* nend, int leaf, const double* cx, const double* cy,
                               const double* cz, const double* cw, const int32_t* cperm,
                               double* nx, double* ny, double* nz, double* nw, int32_t* nperm,
                               double* box, int32_t* nleft, int32_t* choff, double* pbox,
                               int32_t* saxis, double* smid, int32_t* ccnt, int32_t* cleft,
                               hipStream_t s) {
  if (count <= 0) return;
  const dim3 gn((count + WG - 1) / WG), gc(max_chunks);
  hipLaunchKernelGGL(tree_chunk_offsets_kernel, dim3(1), dim3(WG), 0, s, first, count, nbegin,
                     nend, choff);
  hipLaunchKernelGGL(tree_chunk_box_kernel, gc, dim3(WG), 0, s, first, count, choff, nbegin, nend,
                     cx, cy, cz, pbox);
  hipLaunchKernelGGL(tree_node_split_kernel, gn, dim3(WG), 0, s, first, count, choff, nbegin,
                     nend, leaf, pbox, box, saxis, smid);
  hipLaunchKernelGGL(tree_chunk_count_kernel, gc, dim3(WG), 0, s, first, count, choff, nbegin,
                     nend, cx, cy, cz, saxis, smid, ccnt);
  hipLaunchKernelGGL(tree_node_left_kernel, gn, dim3(WG), 0, s, first, count, choff, nbegin,
                     nend, saxis, ccnt, cleft, nleft);
  hipLaunchKernelGGL(tree_chunk_scatter_kernel, gc, dim3(WG), 0, s, first, count, choff, nbegin,
                     nend, saxis, smid, cleft, nleft, cx, cy, cz, cw, cperm, nx, ny, nz, nw, nperm);
  HMX_LAUNCHED();
}

// Children of the split nodes of one level, numbered consecutively after the level.
__global__ void __launch_bounds__(WG) tree_children_kernel(
    int first, int count, int next_first, const int32_t* __restrict__ nleft,
    int32_t* __restrict__ nbegin, int32_t* __restrict__ nend, int32_t* __restrict__ level,
    int32_t* __restrict__ child0, int32_t* __restrict__ child1, int32_t* __restrict__ parent,
    int* next_count) {
  __shared__ int s[NWAVE];
  int run = 0;
  for (int c = 0; c < count; c += WG) {
    int i = c + threadIdx.x;
    int node = first + i;
    bool split = i < count && nleft[node] >= 0;
    int tot;
    int pre = block_excl_scan(split ? 1 : 0, s, &tot);
    if (i < count) {
      if (split) {
        int id0 = next_first + 2 * (run + pre);
        int b = nbegin[node], e = nend[node], nl = nleft[node], lv = level[node];
        child0[node] = id0;
        child1[node] = id0 + 1;
        nbegin[id0] = b;
        nend[id0] = b + nl;
        nbegin[id0 + 1] = b + nl;
        nend[id0 + 1] = e;
        level[id0] = level[id0 + 1] = lv + 1;
        parent[id0] = parent[id0 + 1] = node;
        child0[id0] = child1[id0] = child0[id0 + 1] = child1[id0 + 1] = -1;
      } else {
        child0[node] = child1[node] = -1;
      }
    }
    run += tot;
  }
  if (threadIdx.x == 0) *next_count = 2 * run;
}

void launch_tree_children(int first, int count, int next_first, const int32_t* nleft,
                          int32_t* nbegin, int32_t* nend, int32_t* level, int32_t* child0,
                          int32_t* child1, int32_t* parent, int* next_count, hipStream_t s) {
  hipLaunchKernelGGL(tree_children_kernel, dim3(1), dim3(WG), 0, s, first, count, next_first,
                     nleft, nbegin, nend, level, child0, child1, parent, next_count);
  HMX_LAUNCHED();
}

// Leaves in cluster order: pos_flag[p] = 1 where a leaf begins; start_node[p] = that leaf.
__global__ void leaf_marks_kernel(int n_nodes, const int32_t* __restrict__ nbegin,
                                  const int32_t* __restrict__ child0, int64_t* __restrict__ pos_flag) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n_nodes && child0[i] < 0) pos_flag[nbegin[i]] = 1;
}
void launch_leaf_marks(int n_nodes, const int32_t* nbegin, const int32_t* child0, int64_t* pos_flag,
                       hipStream_t s) {
  hipLaunchKernelGGL(leaf_marks_kernel, dim3((n_nodes + WG - 1) / WG), dim3(WG), 0, s, n_nodes,
                     nbegin, child0, pos_flag);
  HMX_LAUNCHED();
}
__global__ void start_node_kernel(int n_nodes, const int32_t* __restrict__ nbegin,
                                  const int32_t* __restrict__ child0, int32_t* __restrict__ start_node) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n_nodes && child0[i] < 0) start_node[nbegin[i]] = i;
}
void launch_start_node(int n_nodes, const int32_t* nbegin, const int32_t* child0,
                       int32_t* start_node, hipStream_t s) {
  hipLaunchKernelGGL(start_node_kernel, dim3((n_nodes + WG - 1) / WG), dim3(WG), 0, s, n_nodes,
                     nbegin, child0, start_node);
  HMX_LAUNCHED();
}
__global__ void leaf_list_kernel(int64_t M, const int64_t* __restrict__ pos_flag,
                                 const int64_t* __restrict__ pos_scan,
                                 const int32_t* __restrict__ start_node, int32_t* __restrict__ leaves) {
  int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (p < M && pos_flag[p]) leaves[pos_scan[p]] = start_node[p];
}
void launch_leaf_list(int64_t M, const int64_t* pos_flag, const int64_t* pos_scan,
                      const int32_t* start_node, int32_t* leaves, hipStream_t s) {
  hipLaunchKernelGGL(leaf_list_kernel, dim3((unsigned)((M + WG - 1) / WG)), dim3(WG), 0, s, M,
                     pos_flag, pos_scan, start_node, leaves);
  HMX_LAUNCHED();
}
__global__ void leaf_index_kernel(int n_leaves, const int32_t* __restrict__ leaves,
                                  int32_t* __restrict__ leaf_of_node) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n_leaves) leaf_of_node[leaves[i]] = i;
}
void launch_leaf_index(int n_leaves, const int32_t* leaves, int32_t* leaf_of_node, hipStream_t s) {
  hipLaunchKernelGGL(leaf_index_kernel, dim3((n_leaves + WG - 1) / WG), dim3(WG), 0, s, n_leaves,
                     leaves, leaf_of_node);
  HMX_LAUNCHED();
}

}  // namespace hmx

// hmx_build.hip -- build pipeline of an H-matrix operator on the device: cluster tree, block
// tree, near-field blocks, ACA of the far blocks, and the index structures of the product.  The
// host sizes buffers, launches the kernels of the k_*.hip units and moves small index arrays;
// all arithmetic of the operator runs in those kernels.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include <map>
#include <mutex>
#include <utility>

#include "hmx_host.h"
#include "hmx_reg_dev.h"

namespace hmx {
namespace {

// Round to the grid {2^e (1 + j / 8)}: up, or down.
int64_t quantize_up(int64_t n) {
  if (n <= 16) return std::max<int64_t>(n, 1);
  int e = 63 - __builtin_clzll((unsigned long long)n);
  const int64_t step = (int64_t(1) << e) / 8;
  return (n + step - 1) / step * step;
}
int64_t quantize_down(int64_t n) {
  if (n <= 16) return std::max<int64_t>(n, 1);
  int e = 63 - __builtin_clzll((unsigned long long)n);
  const int64_t step = (int64_t(1) << e) / 8;
  return n / step * step;
}

// Grow a device array to `cap` entries keeping the first `keep`.
template <class T>
void grow(DevBuf<T>& b, size_t cap, size_t keep, hipStream_t s) {
  if (b.n >= cap) return;
  DevBuf<T> nb(cap);
  if (keep && b.p) HMX_HIP(hipMemcpyAsync(nb.p, b.p, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipStreamSynchronize(s));
  b = std::move(nb);
}

// HMX_VERBOSE=1 prints the steps of the far-field build with wall-clock times to stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("HMX_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

struct WallLog {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void operator()(const char* what, double a = 0, double b = 0) const {
    if (!verbose()) return;
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[hmx] %9.2f ms  %s %.6g %.6g\n", ms, what, a, b);
  }
};

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    HMX_HIP(hipEventCreate(&a));
    HMX_HIP(hipEventCreate(&b));
    HMX_HIP(hipEventRecord(a, s));
  }
  double stop() {
    HMX_HIP(hipEventRecord(b, s));
    HMX_HIP(hipEventSynchronize(b));
    float ms = 0;
    HMX_HIP(hipEventElapsedTime(&ms, a, b));
    HMX_HIP(hipEventRecord(a, s));
    return ms;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// The two side streams of the ACA classes, created once per device and kept until the process
// ends (default priority, non-blocking).  Created per build, they cost about 0.3 ms a build and
// the second build of a process still ran its classes in the order of a first one (the large
// class last, the phase 1.5 ms longer).  Builds on one device share them; each build joins its
// side-stream work back to its own stream through its own events, so sharing only orders the
// side-stream work of builds that run at the same time.
std::pair<hipStream_t, hipStream_t> aca_side_streams() {
  static std::mutex mu;
  static std::map<int, std::pair<hipStream_t, hipStream_t>> per_dev;
  int dev = 0;
  HMX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = per_dev.find(dev);
  if (it != per_dev.end()) return it->second;
  hipStream_t a = nullptr, b = nullptr;
  HMX_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
  HMX_HIP(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
  per_dev[dev] = {a, b};
  return {a, b};
}

// ------------------------------------------------------------------------------ cluster tree
void build_tree(hmx_op* op, hipStream_t s) {
  const int64_t M = op->M;
  const int leaf = op->p.leaf_size;
  DevBuf<double> bx[2][4];
  DevBuf<int32_t> bp[2];
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < 4; ++c) bx[q][c].alloc(M);
    bp[q].alloc(M);
  }
  // level 0 reads the points in their original order
  HMX_HIP(hipMemcpyAsync(bx[0][0].p, op->X.p, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(bx[0][1].p, op->Y.p, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(bx[0][2].p, op->Z.p, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(bx[0][3].p, op->W.p, M * 8, hipMemcpyDeviceToDevice, s));
  iota_i32(bp[0].p, M, s);

  size_t cap = (size_t)std::max<int64_t>(256, 4 * (M / leaf) + 64);
  DevBuf<int32_t> nbegin(cap), nend(cap), level(cap), child0(cap), child1(cap), parent(cap),
      nleft(cap);
  DevBuf<double> box(6 * cap);
  DevBuf<int> d_next(1);
  // level 0: one root per mesh (a single mesh has one root spanning all points)
  const int nroot = (int)op->mesh_off.size() - 1;
  {
    std::vector<int32_t> rb(nroot), re(nroot), rl(nroot, 0), rp(nroot, -1);
    for (int i = 0; i < nroot; ++i) {
      rb[i] = (int32_t)op->mesh_off[i];
      re[i] = (int32_t)op->mesh_off[i + 1];
    }
    if ((size_t)nroot > cap) {
      cap = 2 * (size_t)nroot;
      for (DevBuf<int32_t>* b : {&nbegin, &nend, &level, &child0, &child1, &parent, &nleft})
        b->alloc(cap);
      box.alloc(6 * cap);
    }
    HMX_HIP(hipMemcpyAsync(nbegin.p, rb.data(), 4 * nroot, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(nend.p, re.data(), 4 * nroot, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(level.p, rl.data(), 4 * nroot, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(parent.p, rp.data(), 4 * nroot, hipMemcpyHostToDevice, s));
    HMX_HIP(hipStreamSynchronize(s));
  }
  int first = 0, count = nroot, total = nroot, cur = 0, depth = 0;
  // scratch of the multi-workgroup level step (levels of at most max_chunked_nodes nodes)
  const int max_chunked_nodes = 1024;
  const int64_t chunk_cap = M / TREE_CHUNK_PTS + max_chunked_nodes + 1;
  DevBuf<int32_t> choff(max_chunked_nodes + 1), saxis(max_chunked_nodes), ccnt(chunk_cap),
      cleft(chunk_cap);
  DevBuf<double> pbox(6 * chunk_cap), smid(max_chunked_nodes);
  // a node splits only if it holds more than `leaf` points, and the nodes of one level are
  // disjoint, so a level adds at most 2 min(count, M / (leaf + 1)) nodes
  const int64_t max_split = M / ((int64_t)leaf + 1);
  while (count > 0) {
    size_t need = (size_t)total + 2 * (size_t)std::min<int64_t>(count, max_split);
    if (need > cap) {
      size_t nc = std::max(need, 2 * cap);
      grow(nbegin, nc, total, s);
      grow(nend, nc, total, s);
      grow(level, nc, total, s);
      grow(child0, nc, total, s);
      grow(child1, nc, total, s);
      grow(parent, nc, total, s);
      grow(nleft, nc, total, s);
      grow(box, 6 * nc, 6 * (size_t)total, s);
      cap = nc;
    }
    const int nx = 1 - cur;
    if (count <= max_chunked_nodes && M >= (int64_t)count * 4 * TREE_CHUNK_PTS) {
      // few large nodes: every node spread over many workgroups
      const int max_chunks = (int)(M / TREE_CHUNK_PTS) + count + 1;
      launch_tree_level_chunked(first, count, max_chunks, nbegin.p, nend.p, leaf, bx[cur][0].p,
                                bx[cur][1].p, bx[cur][2].p, bx[cur][3].p, bp[cur].p, bx[nx][0].p,
                                bx[nx][1].p, bx[nx][2].p, bx[nx][3].p, bp[nx].p, box.p, nleft.p,
                                choff.p, pbox.p, saxis.p, smid.p, ccnt.p, cleft.p, s);
    } else {
      launch_tree_level(first, count, nbegin.p, nend.p, leaf, bx[cur][0].p, bx[cur][1].p,
                        bx[cur][2].p, bx[cur][3].p, bp[cur].p, bx[nx][0].p, bx[nx][1].p,
                        bx[nx][2].p, bx[nx][3].p, bp[nx].p, box.p, nleft.p, s);
    }
    launch_tree_children(first, count, total, nleft.p, nbegin.p, nend.p, level.p, child0.p,
                         child1.p, parent.p, d_next.p, s);
    int next = read1(d_next.p, s);
    first = total;
    total += next;
    count = next;
    cur = nx;
    depth++;
    HMX_REQUIRE(depth < 63, HMX_EUNSUPPORTED, "cluster tree deeper than 62 levels");
  }
  // every leaf range was written to both buffers at the level where it became a leaf
  op->X = std::move(bx[cur][0]);
  op->Y = std::move(bx[cur][1]);
  op->Z = std::move(bx[cur][2]);
  op->W = std::move(bx[cur][3]);
  op->perm = std::move(bp[cur]);
  op->n_nodes = total;
  op->depth = depth;
  op->nbegin = std::move(nbegin);
  op->nend = std::move(nend);
  op->nlevel = std::move(level);
  op->child0 = std::move(child0);
  op->child1 = std::move(child1);
  op->parent = std::move(parent);
  op->box = std::move(box);

  // leaves in cluster order
  DevBuf<int64_t> flag(M), scan(M + 1);
  DevBuf<int32_t> start(M);
  fill_i64(flag.p, 0, M, s);
  launch_leaf_marks(total, op->nbegin.p, op->child0.p, flag.p, s);
  launch_start_node(total, op->nbegin.p, op->child0.p, start.p, s);
  scan_excl_i64(flag.p, scan.p, M, s);
  // the node ranges come back with the leaf count (one wait)
  std::vector<int32_t> hb(total), he(total), hc(total);
  HMX_HIP(hipMemcpyAsync(hb.data(), op->nbegin.p, 4 * (size_t)total, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipMemcpyAsync(he.data(), op->nend.p, 4 * (size_t)total, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipMemcpyAsync(hc.data(), op->child0.p, 4 * (size_t)total, hipMemcpyDeviceToHost, s));
  op->n_leaves = (int)read1(scan.p + M, s);
  op->leaves.alloc(op->n_leaves);
  launch_leaf_list(M, flag.p, scan.p, start.p, op->leaves.p, s);
  op->leaf_of_node.alloc(total);
  fill_i32(op->leaf_of_node.p, -1, total, s);
  launch_leaf_index(op->n_leaves, op->leaves.p, op->leaf_of_node.p, s);
  HMX_HIP(hipStreamSynchronize(s));
  // the product holds one leaf's rows in a workgroup (at most 4 x 64); a leaf can exceed the
  // leaf size only when its points coincide
  op->max_leaf_rows = 0;
  for (int i = 0; i < total; ++i) {
    if (hc[i] >= 0) continue;
    HMX_REQUIRE(he[i] - hb[i] <= 256, HMX_EUNSUPPORTED,
                "a leaf holds more than 256 points (coincident points)");
    op->max_leaf_rows = std::max(op->max_leaf_rows, he[i] - hb[i]);
  }
}

// Sort the near and far lists of (t, s) pairs, each into the lexicographic order of their node
// ranges, with one radix sort: key = (list, rank(t), rank(s)), the ranks in (begin, end) order,
// in ceil(log2(2 n_nodes^2)) bits.
void sort_pairs(hmx_op* op, DevBuf<int2>& nearL, int64_t nn, DevBuf<int2>& farL, int64_t nf,
                hipStream_t s) {
  const int64_t n = nn + nf;
  if (n <= 1) return;
  const int64_t NN = op->n_nodes;
  DevBuf<int64_t> cnt(op->M), start(op->M + 1);
  DevBuf<int32_t> deep(op->M), rank(NN);
  launch_node_rank(op->nbegin.p, op->nlevel.p, (int)NN, op->M, cnt.p, start.p, deep.p, rank.p, s);
  int bits = 1;
  while ((bits < 62) && ((uint64_t)1 << bits) < (uint64_t)NN * (uint64_t)NN) ++bits;
  const uint64_t far_bit = (uint64_t)1 << bits;  // the far list after the near list
  DevBuf<uint64_t> key(n), skey(n);
  DevBuf<int32_t> val(n), sval(n);
  DevBuf<unsigned char> tmp;
  launch_pair_rank_keys(nearL.p, nn, rank.p, NN, 0, 0, key.p, val.p, s);
  launch_pair_rank_keys(farL.p, nf, rank.p, NN, far_bit, nn, key.p, val.p, s);
  radix_sort_u64_pairs(key.p, skey.p, val.p, sval.p, n, bits + 1, tmp, s);
  DevBuf<int2> out_near(std::max<int64_t>(nn, 1)), out_far(std::max<int64_t>(nf, 1));
  launch_pair_gather2(nearL.p, nn, farL.p, sval.p, nn, out_near.p, s);
  launch_pair_gather2(nearL.p, nn, farL.p, sval.p + nn, nf, out_far.p, s);
  HMX_HIP(hipStreamSynchronize(s));
  nearL = std::move(out_near);
  farL = std::move(out_far);
}

// ------------------------------------------------------------------------------ block tree
void build_blocks(hmx_op* op, hipStream_t s) {
  const double eta2 = op->p.eta * op->p.eta;
  // row share: the point range of node number row_share at tree level log2(row_shares)
  int rb = 0, re = (int)op->M;
  if (op->p.row_shares > 1) {
    HMX_REQUIRE(op->mesh_off.size() == 2, HMX_EUNSUPPORTED, "row shares of a batch operator");
    int lev = 0;
    while ((1 << lev) < op->p.row_shares) ++lev;
    std::vector<int32_t> hl, hb, he;
    to_host(hl, op->nlevel.p, op->n_nodes, s);
    to_host(hb, op->nbegin.p, op->n_nodes, s);
    to_host(he, op->nend.p, op->n_nodes, s);
    std::vector<int> at;
    for (int v = 0; v < op->n_nodes; ++v)
      if (hl[v] == lev) at.push_back(v);
    HMX_REQUIRE((int)at.size() == op->p.row_shares, HMX_EUNSUPPORTED,
                "the cluster tree has a leaf above the row-share level");
    rb = hb[at[op->p.row_share]];
    re = he[at[op->p.row_share]];
  }
  op->row_begin = rb;
  op->row_end = re;
  // the frontier starts with (root, root) of every mesh: meshes never interact; an operator
  // between different point sets has the targets' root 0 and the sources' root 1 and starts
  // from (0, 1) only
  const int nroot = op->rect ? 1 : (int)op->mesh_off.size() - 1;
  std::vector<int2> roots(nroot);
  for (int i = 0; i < nroot; ++i) roots[i] = op->rect ? make_int2(0, 1) : make_int2(i, i);
  // Every level descends all non-leaf sides of its pairs, so the recursion ends within the
  // tree's depth: all levels are queued at once and the sizes read back once.  Buffers that
  // turn out too small (the counters still count what was dropped) are enlarged and the
  // recursion runs again.
  const int levels = op->depth;
  HMX_REQUIRE(levels >= 1, HMX_EINTERNAL, "empty cluster tree");
  const int64_t nl = op->n_leaves;
  int64_t fcap = std::max<int64_t>({1024, 32 * nl, 2 * (int64_t)nroot});
  int64_t ncap = std::max<int64_t>(1024, 64 * nl), xcap = std::max<int64_t>(1024, 64 * nl);
  if (op->p.force_block_cap > 0) {
    fcap = std::max<int64_t>(op->p.force_block_cap, nroot);
    ncap = xcap = op->p.force_block_cap;
  }
  // counters: [L] pairs after level L, [levels] near, [levels + 1] far, [levels + 2] error
  // bits, [levels + 3] the roots
  DevBuf<int> cnt(levels + 4);
  std::vector<int> c(levels + 4);
  DevBuf<int2> buf[2], nearL, farL;
  for (int attempt = 0;; ++attempt) {
    HMX_REQUIRE(attempt < 64, HMX_EINTERNAL, "block recursion buffers did not converge");
    buf[0].alloc(fcap);
    buf[1].alloc(fcap);
    nearL.alloc(ncap);
    farL.alloc(xcap);
    fill_i32(cnt.p, 0, levels + 3, s);
    fill_i32(cnt.p + levels + 3, nroot, 1, s);
    HMX_HIP(hipMemcpyAsync(buf[0].p, roots.data(), sizeof(int2) * nroot, hipMemcpyHostToDevice,
                           s));
    for (int L = 0; L < levels; ++L)
      launch_block_level(buf[L & 1].p, L == 0 ? cnt.p + levels + 3 : cnt.p + L - 1, fcap,
                         op->box.p, op->child0.p, op->child1.p, op->nbegin.p, op->nend.p, rb, re,
                         eta2, op->p.max_far_mn, buf[(L + 1) & 1].p, fcap, cnt.p + L, nearL.p,
                         ncap, cnt.p + levels, farL.p, xcap, cnt.p + levels + 1,
                         cnt.p + levels + 2, s);
    HMX_HIP(hipMemcpyAsync(c.data(), cnt.p, sizeof(int) * (levels + 3), hipMemcpyDeviceToHost, s));
    HMX_HIP(hipStreamSynchronize(s));
    const int err = c[levels + 2];
    HMX_REQUIRE((err & 1) == 0, HMX_EUNSUPPORTED,
                "a block crosses the row-share boundary (use fewer row shares)");
    if (err & 2) {
      int64_t fmax = 0;
      for (int L = 0; L < levels; ++L) fmax = std::max<int64_t>(fmax, c[L]);
      fcap = std::max<int64_t>(2 * fcap, 2 * fmax);
      ncap = std::max<int64_t>(2 * ncap, 2 * (int64_t)c[levels]);
      xcap = std::max<int64_t>(2 * xcap, 2 * (int64_t)c[levels + 1]);
      continue;
    }
    HMX_REQUIRE(c[levels - 1] == 0, HMX_EINTERNAL, "block recursion deeper than the cluster tree");
    break;
  }
  op->n_near = c[levels];
  op->n_far = c[levels + 1];
  sort_pairs(op, nearL, op->n_near, farL, op->n_far, s);
  op->nearL = std::move(nearL);
  op->farL = std::move(farL);
}

// ------------------------------------------------------------------------------ near field
template <class T>
void build_near(hmx_op* op, hipStream_t s) {
  const int64_t nn = op->n_near;
  const int nl = op->n_leaves;
  op->near_tb.alloc(std::max<int64_t>(nn, 1));
  op->near_m.alloc(std::max<int64_t>(nn, 1));
  op->near_sb.alloc(std::max<int64_t>(nn, 1));
  op->near_n.alloc(std::max<int64_t>(nn, 1));
  DevBuf<int64_t> sizes(std::max<int64_t>(nn, 1)), lcnt(nl);
  op->near_off.alloc(nn + 1);
  op->near_ptr.alloc(nl + 1);
  fill_i64(lcnt.p, 0, nl, s);
  launch_pair_ranges(op->nearL.p, nn, op->nbegin.p, op->nend.p, op->near_tb.p, op->near_m.p,
                     op->near_sb.p, op->near_n.p, s);
  launch_near_prep(op->nearL.p, nn, op->nbegin.p, op->nend.p, op->leaf_of_node.p, sizes.p, lcnt.p, s);
  scan_excl_i64(sizes.p, op->near_off.p, nn, s);
  scan_excl_i64(lcnt.p, op->near_ptr.p, nl, s);
  op->near_entries = read1(op->near_off.p + nn, s);
  if (op->p.near_mode == 1) return;  // the product evaluates the near blocks itself
  size_t bytes = (size_t)op->near_entries * sizeof(T);
  if (op->p.pool_limit_bytes > 0 && (int64_t)bytes > op->p.pool_limit_bytes)
    throw Error(HMX_ENOMEM, "near field exceeds pool_limit_bytes");
  op->near_pool.alloc(std::max<size_t>(bytes, 1));
  // the singular correction of close pairs (Section 5.2) goes into the near field only
  RegArgs ra{};
  DevBuf<int32_t> iperm;
  if (op->reg) {
    iperm.alloc(op->M);
    launch_iperm(op->perm.p, op->M, iperm.p, s);
    ra.perm = op->perm.p;
    ra.iperm = iperm.p;
    ra.tgeo = op->tgeo.p;
    std::copy(op->reg_lag, op->reg_lag + 9, ra.lag);
  }
  launch_assemble<T>(op->near_tb.p, op->near_m.p, op->near_sb.p, op->near_n.p, op->near_off.p, nn,
                     op->X.p, op->Y.p, op->Z.p, op->W.p, op->kern, op->kpt.p, (T*)op->near_pool.p,
                     op->reg ? &ra : nullptr, s);
  HMX_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------ far field
template <class T>
void build_far(hmx_op* op, hipStream_t s) {
  WallLog wl;
  const int64_t nf = op->n_far;
  const int nl = op->n_leaves;
  const int64_t nf1 = std::max<int64_t>(nf, 1);
  DevBuf<int32_t> ftb(nf1), fm(nf1), fsb(nf1), fn(nf1);
  DevBuf<int64_t> node_cnt(op->n_nodes);
  DevBuf<int32_t> node_first(op->n_nodes);
  fill_i64(node_cnt.p, 0, op->n_nodes, s);
  fill_i32(node_first.p, -1, op->n_nodes, s);
  launch_far_prep(op->farL.p, nf, op->nbegin.p, op->nend.p, ftb.p, fm.p, fsb.p, fn.p, node_cnt.p,
                  node_first.p, s);

  // descriptors on the device: rank cap, first slot size, used-flag offsets, pool estimate,
  // scheduling key (slots are taken from the device pool by the kernels)
  DevBuf<FarDesc> d_desc(nf1);
  DevBuf<int64_t> mnv(nf1), foff(nf1 + 1), estv(nf1), ests(nf1 + 1), work(nf1);
  DevBuf<uint8_t> wave(nf1);
  launch_far_desc(op->farL.p, nf, op->nbegin.p, op->nend.p, op->p.initial_rank,
                  op->p.force_rank_cap, op->p.aca_wave, d_desc.p, mnv.p, estv.p, wave.p, work.p, s);
  scan_excl_i64(mnv.p, foff.p, nf, s);
  scan_excl_i64(estv.p, ests.p, nf, s);
  launch_far_foff(d_desc.p, foff.p, nf, s);
  int64_t sums[2] = {0, 0};  // used-flag bytes, pool estimate
  HMX_HIP(hipMemcpyAsync(&sums[0], foff.p + nf, 8, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipMemcpyAsync(&sums[1], ests.p + nf, 8, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipStreamSynchronize(s));
  const int64_t flag_bytes = sums[0];
  int64_t sum_mn = sums[1];
  // learned layout: the slot pool is reserved from the predicted ranks r_alloc (checked against
  // the device memory before ACA runs) instead of the generic estimate, and the scheduling key
  // becomes the predicted work r_alloc^2 (m + n); blocks that outgrow their prediction take the
  // room others leave
  if (op->p.rank_model == HMX_RANK_LEARNED && nf > 0) {
    const RankModel rm = get_rank_model();
    HMX_REQUIRE(rm.set, HMX_EINVAL, "rank_model is learned but no model was set (hmx_set_rank_model)");
    DevBuf<float> feat(4 * nf), pred(nf), th(MLP_NPARAMS), nm(8);
    DevBuf<int64_t> ramn(nf1), rsum(nf1 + 1);
    HMX_HIP(hipMemcpyAsync(th.p, rm.theta, MLP_NPARAMS * 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(nm.p, rm.norm, 8 * 4, hipMemcpyHostToDevice, s));
    launch_mlp_features(op->farL.p, nf, op->nbegin.p, op->nend.p, op->box.p, op->kpt.p, feat.p, s);
    launch_mlp_predict(th.p, nm.p, feat.p, nf, pred.p, s);
    launch_far_pred(pred.p, d_desc.p, nf, rm.alpha, (int64_t)std::lround(rm.beta),
                    op->p.force_pred_scale, ramn.p, work.p, s);
    scan_excl_i64(ramn.p, rsum.p, nf, s);
    const int64_t total = read1(rsum.p + nf, s);
    size_t fb = 0, tb = 0;
    HMX_HIP(hipMemGetInfo(&fb, &tb));
    fb += dev_cached_bytes();
    HMX_REQUIRE((double)total * sizeof(T) <= 0.9 * (double)fb, HMX_ENOMEM,
                "predicted factor storage exceeds the free device memory");
    sum_mn = std::max<int64_t>(total, (int64_t)(64 << 20) / (int64_t)sizeof(T));
    op->predicted_entries = total;
  }
  // launch order of the first round: by class, then by decreasing floor(log2(work))
  const int64_t big_mn = op->p.aca_big_mn, small_mn = op->p.aca_small_mn;
  DevBuf<int32_t> d_order(nf1);
  DevBuf<int> key_hist(FAR_ORDER_KEYS), key_cursor(FAR_ORDER_KEYS);
  launch_far_order(d_desc.p, wave.p, work.p, nf, big_mn, small_mn, key_hist.p, key_cursor.p,
                   d_order.p, s);
  int class_count[4] = {0, 0, 0, 0};
  {
    std::vector<int> hh;
    to_host(hh, key_hist.p, nf > 0 ? FAR_ORDER_KEYS : 0, s);
    for (size_t q = 0; q < hh.size(); ++q) class_count[q / 64] += hh[q];
  }
  // arenas of the two workgroup classes: at most ACA_ARENA_* entries, and no more than a quarter
  // of each workgroup's share of the estimate (small problems take small arenas); each
  // workgroup may leave the unused rest of one arena, which the pool provides for
  const int mid_threads = op->p.aca_mid_threads;
  const int big_threads = op->p.aca_big_threads;
  const int64_t grid_big = aca_grid<T>(big_threads, ACA_KIND_BIG);
  const int64_t grid_mid = aca_grid<T>(mid_threads, ACA_KIND_MID);
  const int64_t grid_small = aca_grid<T>(64, ACA_KIND_SMALL);
  int64_t arena_big = 0, arena_mid = 0, arena_small = 0;
  if (op->p.aca_arena) {
    const int64_t share = sum_mn / (4 * (grid_big + grid_mid + grid_small));
    arena_big = std::min<int64_t>(ACA_ARENA_BIG, std::max<int64_t>(share, 1));
    arena_mid = std::min<int64_t>(ACA_ARENA_MID, std::max<int64_t>(share, 1));
    arena_small = std::min<int64_t>(ACA_ARENA_SMALL, std::max<int64_t>(share, 1));
    sum_mn += grid_big * arena_big + grid_mid * arena_mid + grid_small * arena_small;
  }
  // device pool for factor slots, within the free memory
  size_t free_b = 0, total_b = 0;
  HMX_HIP(hipMemGetInfo(&free_b, &total_b));
  free_b += dev_cached_bytes();  // blocks held by the library's cache are free for its use
  // sizes on a grid of 1/8 octave, so that a repeated build asks the allocator's cache for the
  // same size again instead of a slightly different one
  const int64_t min_pool = (int64_t)(64 << 20) / (int64_t)sizeof(T);
  int64_t gcap = std::min<int64_t>(quantize_up(std::max<int64_t>(sum_mn, min_pool)),
                                   quantize_down((int64_t)(0.6 * (double)free_b) / (int64_t)sizeof(T)));
  if (op->p.force_pool_bytes > 0) gcap = op->p.force_pool_bytes / (int64_t)sizeof(T);
  gcap = std::max<int64_t>(gcap, 1);
  wl("descriptors built: blocks, pool entries", (double)nf, (double)gcap);
  DevBuf<T> gpool;
  gpool.alloc_block(gcap);  // trimmed after ACA: a block of its own
  op->pool_reserved_bytes = gcap * (int64_t)sizeof(T);
  wl("pool allocated (GiB)", (double)gcap * sizeof(T) / (1 << 30));
  DevBuf<uint8_t> flags(std::max<int64_t>(flag_bytes, 1));
  DevBuf<int32_t> rank(nf1), ipiv(nf1), status(nf1);
  DevBuf<double> norm2(nf1);
  DevBuf<int> counter(3);
  DevBuf<unsigned long long> gtop(1);
  fill_i64((int64_t*)gtop.p, 0, 1, s);

  wl("device state ready");
  // side streams for the block classes (default priority), joined back to `s`
  const auto side = aca_side_streams();
  hipStream_t s2_ = side.first, s3_ = side.second;
  hipEvent_t ev_ready = nullptr, ev_d2 = nullptr, ev_d3 = nullptr;
  struct EvGuard {
    hipEvent_t* ev[3];
    ~EvGuard() {
      for (auto e : ev)
        if (*e) (void)hipEventDestroy(*e);
    }
  } guard{{&ev_ready, &ev_d2, &ev_d3}};
  HMX_HIP(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
  HMX_HIP(hipEventCreateWithFlags(&ev_d2, hipEventDisableTiming));
  HMX_HIP(hipEventCreateWithFlags(&ev_d3, hipEventDisableTiming));
  // timing of each class's first launch, on the stream it runs on
  hipEvent_t tev[8] = {};
  struct EventGuard {
    hipEvent_t* e;
    ~EventGuard() {
      for (int i = 0; i < 8; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } tguard{tev};
  for (auto& e : tev) HMX_HIP(hipEventCreate(&e));
  // Gram scratch of the three workgroup classes: 2 order^2 entries per workgroup
  auto gram_entries = [](int64_t grid, int threads, int kind) {
    const int64_t g = aca_gram_order(threads, kind);
    return (size_t)(grid * 2 * g * g);
  };
  DevBuf<double2> gram_big(gram_entries(grid_big, big_threads, ACA_KIND_BIG));
  DevBuf<double2> gram_mid(gram_entries(grid_mid, mid_threads, ACA_KIND_MID));
  DevBuf<double2> gram_small(gram_entries(grid_small, 64, ACA_KIND_SMALL));
  // blocks below aca_gram_min_mn take the direct cross sums (fewer barriers per step)
  const int gram_min = op->p.aca_gram_min_mn;

  // host copies for the rounds that continue blocks (filled only if a round is needed)
  std::vector<FarDesc> desc;
  std::vector<uint8_t> is_wave;
  std::vector<int64_t> est, hwork;
  // run ACA with the classes of (nbig, nmid, nwave, nsmall) blocks laid out in that order in
  // d_order: m + n >= aca_big_mn in aca_big_threads-thread workgroups (stream s2), m, n <=
  // ACA_WAVE_N one per wavefront (stream s3, blocks that have not started), then the small
  // blocks (m + n < aca_small_mn) in 64-thread workgroups (stream s3), the others in
  // aca_mid_threads-thread workgroups (stream s)
  auto launch_round = [&](int nbig, int nmid, int nwave, int nsmall, int fresh) {
    fill_i32(counter.p, 0, 3, s);
    // aca_serial = 1 runs the classes one after the other on `s` (same work; also used to time
    // each class on its own)
    const bool serial = op->p.aca_serial != 0;
    hipStream_t s2 = serial ? s : s2_;
    hipStream_t s3 = serial ? s : s3_;
    HMX_HIP(hipEventRecord(ev_ready, s));
    HMX_HIP(hipStreamWaitEvent(s2, ev_ready, 0));
    HMX_HIP(hipStreamWaitEvent(s3, ev_ready, 0));
    if (fresh) HMX_HIP(hipEventRecord(tev[0], s2));
    launch_aca<T>(d_desc.p, d_order.p, nbig, counter.p, big_threads, ACA_KIND_BIG, op->X.p, op->Y.p, op->Z.p,
                  op->W.p, op->kern, op->kpt.p, op->p.tol, flags.p, rank.p, ipiv.p, status.p, norm2.p,
                  fresh, gpool.p, gcap, gtop.p, gram_big.p, gram_min, arena_big, s2);
    if (fresh) HMX_HIP(hipEventRecord(tev[1], s2));
    if (fresh) HMX_HIP(hipEventRecord(tev[4], s3));
    launch_aca_wave<T>(d_desc.p, d_order.p + nbig + nmid, nwave, op->X.p,
                       op->Y.p, op->Z.p, op->W.p, op->kern, op->kpt.p, op->p.tol, flags.p, rank.p,
                       ipiv.p, status.p, norm2.p, gpool.p, gcap, gtop.p, s3);
    if (fresh) HMX_HIP(hipEventRecord(tev[5], s3));
    if (fresh) HMX_HIP(hipEventRecord(tev[6], s3));
    launch_aca<T>(d_desc.p, d_order.p + nbig + nmid + nwave, nsmall, counter.p + 2, 64,
                  ACA_KIND_SMALL, op->X.p, op->Y.p, op->Z.p, op->W.p, op->kern, op->kpt.p,
                  op->p.tol, flags.p, rank.p, ipiv.p, status.p, norm2.p, fresh, gpool.p, gcap,
                  gtop.p, gram_small.p, gram_min, arena_small, s3);
    if (fresh) HMX_HIP(hipEventRecord(tev[7], s3));
    if (fresh) HMX_HIP(hipEventRecord(tev[2], s));
    launch_aca<T>(d_desc.p, d_order.p + nbig, nmid, counter.p + 1, mid_threads, ACA_KIND_MID,
                  op->X.p,
                  op->Y.p, op->Z.p, op->W.p, op->kern, op->kpt.p, op->p.tol, flags.p, rank.p, ipiv.p,
                  status.p, norm2.p, fresh, gpool.p, gcap, gtop.p, gram_mid.p, gram_min, arena_mid,
                  s);
    if (fresh) HMX_HIP(hipEventRecord(tev[3], s));
    HMX_HIP(hipEventRecord(ev_d2, s2));
    HMX_HIP(hipEventRecord(ev_d3, s3));
    HMX_HIP(hipStreamWaitEvent(s, ev_d2, 0));
    HMX_HIP(hipStreamWaitEvent(s, ev_d3, 0));
    HMX_HIP(hipStreamSynchronize(s));
  };
  // a later round: the listed blocks ordered on the host like the first round, with the
  // wavefront class for the blocks that have not started (`started`: ranks before the round)
  auto run_list = [&](const std::vector<int32_t>& list, const std::vector<int32_t>& started) {
    std::vector<int32_t> bucket[4][64];
    for (int32_t b : list) {
      const FarDesc& d = desc[b];
      const int64_t mn = (int64_t)d.m + d.n;
      const int cls = mn >= big_mn                        ? 0
                      : (started[b] == 0 && is_wave[b])   ? 2
                      : (mn < small_mn && d.rcap <= ACA_COEF_SMALL) ? 3
                                                          : 1;
      const int lw = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(hwork[b], 1));
      bucket[cls][63 - lw].push_back(b);
    }
    std::vector<int32_t> ord;
    int cnt[4] = {0, 0, 0, 0};
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < 64; ++q) {
        ord.insert(ord.end(), bucket[c][q].begin(), bucket[c][q].end());
        cnt[c] += (int)bucket[c][q].size();
      }
    if (!ord.empty())
      HMX_HIP(hipMemcpyAsync(d_order.p, ord.data(), ord.size() * 4, hipMemcpyHostToDevice, s));
    launch_round(cnt[0], cnt[1], cnt[2], cnt[3], 0);
  };
  {
    wl("first launch start");
    launch_round(class_count[0], class_count[1], class_count[2], class_count[3], 1);
    wl("first launch done");
    for (int c = 0; c < 4; ++c) {
      float ms = 0.f;
      HMX_HIP(hipEventElapsedTime(&ms, tev[2 * c], tev[2 * c + 1]));
      op->aca_ms[c] = ms;
    }
  }
  op->aca_rounds = 1;
  // Blocks stopped with OVERFLOW (device pool exhausted, or a wavefront block past its register
  // capacity) continue in further rounds, each with a new pool sized from the estimates of the
  // blocks left (the old pools keep the finished factors).  A block resumes from its saved state
  // and takes its slots from the new pool in the kernel; one that had not started runs as a
  // fresh block.  The first launch's statuses are summarised on the device; the host reads the
  // per-block state only when a round is needed.
  std::vector<DevBuf<T>> old_pools;
  int64_t used_old = 0;  // entries taken from pools already retired
  DevBuf<uint8_t> d_cont;  // blocks continued in a later round (allocated with the first round)
  DevBuf<int> nover(1);
  launch_count_status(status.p, nf, ACA_OVERFLOW, nover.p, s);
  if (nf > 0 && read1(nover.p, s) > 0) {
    std::vector<int32_t> hst, hrank, first_cap(nf);
    std::vector<uint8_t> continued(nf, 0);
    to_host(desc, d_desc.p, nf, s);
    to_host(is_wave, wave.p, nf, s);
    to_host(est, estv.p, nf, s);
    to_host(hwork, work.p, nf, s);
    to_host(hst, status.p, nf, s);
    for (int64_t b = 0; b < nf; ++b) first_cap[b] = desc[b].cap + desc[b].cap1;
    for (;;) {
      std::vector<int32_t> list;
      for (int64_t b = 0; b < nf; ++b)
        if ((hst[b] & 0xff) == ACA_OVERFLOW) list.push_back((int32_t)b);
      if (list.empty()) break;
      to_host(hrank, rank.p, nf, s);
      to_host(desc, d_desc.p, nf, s);  // current slots (moved on the device)
      int64_t need = 0;
      for (int32_t b : list) {
        continued[b] = 1;
        // room to finish: a doubled slot, at least twice the rank reached so far
        const int64_t c = std::max<int64_t>({(int64_t)desc[b].cap + desc[b].cap1, (int64_t)hrank[b] + 8,
                                             (int64_t)first_cap[b]});
        need += std::max<int64_t>(est[b], 2 * c * ((int64_t)desc[b].m + desc[b].n));
      }
      // each workgroup that takes a block may leave the unused rest of one arena
      need += std::min<int64_t>((int64_t)list.size(), grid_big + grid_mid + grid_small) *
              std::max({arena_big, arena_mid, arena_small});
      HMX_HIP(hipMemGetInfo(&free_b, &total_b));
      free_b += dev_cached_bytes();
      int64_t ncap = std::min<int64_t>(quantize_up(std::max<int64_t>(need, min_pool)),
                                       quantize_down((int64_t)(0.6 * (double)free_b) / (int64_t)sizeof(T)));
      HMX_REQUIRE(ncap > 0, HMX_ENOMEM, "device memory exhausted during ACA");
      const int64_t top = std::min<int64_t>((int64_t)read1(gtop.p, s), gcap);
      used_old += top;
      wl("round: blocks left, new pool entries", (double)list.size(), (double)ncap);
      gpool.shrink(top);  // the retired pool keeps the slots it handed out
      old_pools.push_back(std::move(gpool));
      gpool.alloc_block(ncap);
      op->pool_reserved_bytes += ncap * (int64_t)sizeof(T);
      wl("round: pool allocated");
      gcap = ncap;
      fill_i64((int64_t*)gtop.p, 0, 1, s);
      const std::vector<int32_t> before = hrank;
      run_list(list, before);
      wl("round: launch done");
      op->aca_rounds++;
      to_host(hst, status.p, nf, s);
      to_host(hrank, rank.p, nf, s);
      bool progress = false;
      for (int32_t b : list)
        if ((hst[b] & 0xff) != ACA_OVERFLOW || hrank[b] != before[b]) progress = true;
      HMX_REQUIRE(progress, HMX_ENOMEM, "device memory exhausted during ACA (no block progressed)");
    }
    d_cont.alloc(nf);
    HMX_HIP(hipMemcpyAsync(d_cont.p, continued.data(), nf, hipMemcpyHostToDevice, s));
  }

  wl("ACA finished");
  // records of the product: factors stay in the slots ACA wrote; dense blocks are assembled
  op->far.alloc(nf1);
  DevBuf<int64_t> tcnt(nf1), toff(nf1 + 1), dcnt(nf1), doff(nf1 + 1), dflg(nf1), dpos(nf1 + 1);
  DevBuf<unsigned long long> stats(FAR_STATS);
  DevBuf<int> bad(1);
  fill_i64((int64_t*)stats.p, 0, FAR_STATS, s);
  fill_i32(bad.p, 0, 1, s);
  launch_far_rec(d_desc.p, rank.p, status.p, d_cont.p, wave.p, big_mn, small_mn, (int)sizeof(T), nf,
                 op->far.p, tcnt.p, dcnt.p, dflg.p, stats.p, bad.p, s);
  scan_excl_i64(tcnt.p, toff.p, nf, s);
  scan_excl_i64(dcnt.p, doff.p, nf, s);
  scan_excl_i64(dflg.p, dpos.p, nf, s);
  struct {
    unsigned long long st[FAR_STATS];
    int64_t t_len, drun, nd, used;
    int bad;
  } h{};
  HMX_HIP(hipMemcpyAsync(h.st, stats.p, sizeof(h.st), hipMemcpyDeviceToHost, s));
  if (nf > 0) {
    HMX_HIP(hipMemcpyAsync(&h.t_len, toff.p + nf, 8, hipMemcpyDeviceToHost, s));
    HMX_HIP(hipMemcpyAsync(&h.drun, doff.p + nf, 8, hipMemcpyDeviceToHost, s));
    HMX_HIP(hipMemcpyAsync(&h.nd, dpos.p + nf, 8, hipMemcpyDeviceToHost, s));
  }
  HMX_HIP(hipMemcpyAsync(&h.used, gtop.p, 8, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipMemcpyAsync(&h.bad, bad.p, 4, hipMemcpyDeviceToHost, s));
  HMX_HIP(hipStreamSynchronize(s));
  HMX_REQUIRE(!h.bad, HMX_EINTERNAL, "ACA left a block unfinished");
  op->far_entries = (int64_t)h.st[0];
  op->sum_rank = (int64_t)h.st[1];
  op->max_rank = (int64_t)h.st[2];
  op->dense_far = (int64_t)h.st[3];
  op->dense_far_entries = (int64_t)h.st[4];
  op->overflow_blocks = (int64_t)h.st[5];
  op->kernel_evals += (int64_t)h.st[6];
  // per class: blocks, and the bytes ACA must move: step k reads the k previous columns of U
  // and V once (residual row and column) and writes one column pair, so a block of final rank r
  // moves es (m + n) r (r + 1) / 2 bytes
  for (int c = 0; c < 4; ++c) {
    op->aca_blocks[c] = (int64_t)h.st[7 + c];
    op->aca_bytes[c] = (int64_t)h.st[11 + c];
  }
  op->t_len = h.t_len;
  op->pool_used_bytes = (std::min(h.used, gcap) + used_old) * (int64_t)sizeof(T);
  op->dense_pool.alloc(std::max<int64_t>(h.drun, 1) * sizeof(T));
  if (op->p.pool_limit_bytes > 0 &&
      op->pool_used_bytes + (int64_t)op->near_pool.bytes() + (int64_t)op->dense_pool.bytes() >
          op->p.pool_limit_bytes)
    throw Error(HMX_ENOMEM, "operator exceeds pool_limit_bytes");
  {
    const int64_t nd = std::max<int64_t>(h.nd, 1);
    DevBuf<int32_t> dtb(nd), dm(nd), dsb(nd), dn(nd);
    DevBuf<int64_t> dofs(nd);
    launch_far_rec_finish<T>(op->far.p, toff.p, doff.p, dpos.p, nf, (T*)op->dense_pool.p, dtb.p,
                             dm.p, dsb.p, dn.p, dofs.p, s);
    if (h.nd > 0)
      launch_assemble<T>(dtb.p, dm.p, dsb.p, dn.p, dofs.p, h.nd, op->X.p, op->Y.p, op->Z.p,
                         op->W.p, op->kern, op->kpt.p, (T*)op->dense_pool.p, nullptr, s);
    HMX_HIP(hipStreamSynchronize(s));
  }
  // keep the pools (they hold the factors), trimmed to the slots handed out: the reserve above
  // them goes back to the allocator
  gpool.shrink(std::min(h.used, gcap));
  op->far_pools.clear();
  {
    DevBuf<unsigned char> g;
    g.p = (unsigned char*)gpool.p;
    g.n = gpool.bytes();
    gpool.p = nullptr;
    gpool.n = 0;
    op->far_pools.push_back(std::move(g));
    for (auto& p : old_pools) {
      DevBuf<unsigned char> e;
      e.p = (unsigned char*)p.p;
      e.n = p.bytes();
      p.p = nullptr;
      p.n = 0;
      op->far_pools.push_back(std::move(e));
    }
  }
  wl("records and dense far blocks done");

  wl("far records on device");
  // per leaf: far blocks whose row node contains it
  DevBuf<int64_t> lcnt(nl);
  op->far_ptr.alloc(nl + 1);
  launch_leaf_far_count(nl, op->leaves.p, op->parent.p, node_cnt.p, lcnt.p, s);
  scan_excl_i64(lcnt.p, op->far_ptr.p, nl, s);
  int64_t ninc = read1(op->far_ptr.p + nl, s);
  op->far_list.alloc(std::max<int64_t>(ninc, 1));
  launch_leaf_far_fill(nl, op->leaves.p, op->parent.p, node_cnt.p, node_first.p, op->far_ptr.p,
                       op->far_list.p, s);
  HMX_HIP(hipStreamSynchronize(s));
  wl("per-leaf far lists done");
}

template <class T>
void build_h(hmx_op* op, hipStream_t s) {
  HMX_REQUIRE(op->M < (int64_t(1) << 23), HMX_EUNSUPPORTED,
              "H-matrix mode supports at most 2^23 - 1 points");
  Timer tm(s);
  Timer total(s);
  build_tree(op, s);
  op->t_tree = tm.stop();
  build_blocks(op, s);
  op->t_blocks = tm.stop();
  build_near<T>(op, s);
  if (op->p.near_mode == 0) op->kernel_evals += op->near_entries;
  op->t_near = tm.stop();
  build_far<T>(op, s);
  op->t_aca = tm.stop();
  op->xp.alloc((size_t)op->M * sizeof(T));
  op->tbuf.alloc(std::max<size_t>((size_t)op->t_len * sizeof(T), sizeof(T)));
  op->t_total = total.stop();
}

}  // namespace

void finish_build(hmx_op* op, hipStream_t s) {
  const size_t es = op->prec == HMX_FP64 ? sizeof(double2) : sizeof(float2);
  op->elem = es;
  if (op->mesh_off.empty()) {
    op->mesh_off = {0, op->M};
    op->mesh_k = {op->k};
  }
  HMX_REQUIRE(op->mesh_off.back() == op->M, HMX_EINTERNAL, "mesh offsets do not cover the points");
  if (!op->rect) {
    op->rows = op->cols = op->M;
    op->x_off = 0;
  }
  op->kpt.alloc(op->M);
  for (size_t i = 0; i + 1 < op->mesh_off.size(); ++i)
    fill_f64(op->kpt.p + op->mesh_off[i], op->mesh_k[i], op->mesh_off[i + 1] - op->mesh_off[i], s);
  if (op->p.tol <= 0) {
    op->dense = true;
    op->partial.alloc((size_t)dense_otf_partial_len(op->rows, op->cols) * es);
    return;
  }
  if (op->prec == HMX_FP64) build_h<double2>(op, s);
  else build_h<float2>(op, s);
}

}  // namespace hmx

// hmx_api.hip -- the C ABI of libhmx: argument checks, build orchestration, product dispatch,
// queries.  All arithmetic of the operator runs in the kernels of the k_*.hip units; this file
// only sizes buffers, launches kernels and moves small index arrays.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hmx_host.h"

using namespace hmx;

namespace {

thread_local std::string g_err;

hmx_status fail(hmx_status c, const std::string& m) {
  g_err = m;
  return c;
}

#define API_TRY try {
#define API_CATCH                                            \
  }                                                          \
  catch (const hmx::Error& e) {                              \
    return fail(e.code, e.what());                           \
  }                                                          \
  catch (const std::bad_alloc&) {                            \
    return fail(HMX_ENOMEM, "host allocation failed");       \
  }                                                          \
  catch (const std::exception& e) {                          \
    return fail(HMX_EINTERNAL, e.what());                    \
  }

void defaults(hmx_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->struct_size = (int32_t)sizeof(hmx_params);
  p->tol = 1e-3;
  p->leaf_size = 64;
  p->eta = 1.5;
  p->precision = HMX_FP64;
  p->rank_model = HMX_RANK_ADAPTIVE;
  p->initial_rank = 16;
  p->force_pred_scale = 1.0;
  p->force_rank_cap = 0;
  p->pool_limit_bytes = 0;
}

hmx_params resolve(const hmx_params* in) {
  hmx_params p;
  defaults(&p);
  if (in) {
    HMX_REQUIRE(in->struct_size == (int32_t)sizeof(hmx_params), HMX_EINVAL,
                "hmx_params.struct_size does not match this library (use hmx_params_default)");
    p = *in;
  }
  HMX_REQUIRE(std::isfinite(p.tol), HMX_EINVAL, "tol must be finite");
  HMX_REQUIRE(p.leaf_size >= 1, HMX_EINVAL, "leaf_size must be >= 1");
  HMX_REQUIRE(p.leaf_size <= 256, HMX_EUNSUPPORTED, "leaf_size above 256 is not supported");
  HMX_REQUIRE(std::isfinite(p.eta) && p.eta > 0, HMX_EINVAL, "eta must be finite and > 0");
  HMX_REQUIRE(p.precision == HMX_FP64 || p.precision == HMX_FP32_MIXED, HMX_EINVAL,
              "unknown precision");
  HMX_REQUIRE(p.rank_model == HMX_RANK_ADAPTIVE || p.rank_model == HMX_RANK_LEARNED, HMX_EINVAL,
              "unknown rank_model");
  HMX_REQUIRE(p.initial_rank >= 1, HMX_EINVAL, "initial_rank must be >= 1");
  HMX_REQUIRE(std::isfinite(p.force_pred_scale) && p.force_pred_scale >= 0, HMX_EINVAL,
              "force_pred_scale must be finite and >= 0");
  HMX_REQUIRE(p.force_rank_cap >= 0, HMX_EINVAL, "force_rank_cap must be >= 0");
  HMX_REQUIRE(p.pool_limit_bytes >= 0, HMX_EINVAL, "pool_limit_bytes must be >= 0");
  return p;
}

Rule make_rule(const double* q_bary, const double* q_w, int32_t nq) {
  HMX_REQUIRE(q_bary && q_w, HMX_EINVAL, "null quadrature rule");
  HMX_REQUIRE(nq >= 1, HMX_EINVAL, "n_q must be >= 1");
  HMX_REQUIRE(nq <= MAX_NQ, HMX_EUNSUPPORTED, "n_q above 32 is not supported");
  Rule r{};
  r.nq = nq;
  double ws = 0.0;
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) {
      double l = q_bary[3 * q + j];
      HMX_REQUIRE(std::isfinite(l) && l >= -1e-12, HMX_EINVAL,
                  "barycentric coordinates must lie in the triangle");
      r.b[q][j] = l;
      s += l;
    }
    HMX_REQUIRE(std::fabs(s - 1.0) <= 1e-12, HMX_EINVAL, "barycentric coordinates must sum to 1");
    HMX_REQUIRE(std::isfinite(q_w[q]), HMX_EINVAL, "non-finite quadrature weight");
    r.w[q] = q_w[q];
    ws += q_w[q];
  }
  HMX_REQUIRE(std::fabs(ws - 1.0) <= 1e-12, HMX_EINVAL, "reference weights must sum to 1");
  return r;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
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
  {
    int32_t root[4] = {0, (int32_t)M, 0, -1};
    HMX_HIP(hipMemcpyAsync(nbegin.p, &root[0], 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(nend.p, &root[1], 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(level.p, &root[2], 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(parent.p, &root[3], 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipStreamSynchronize(s));
  }
  int first = 0, count = 1, total = 1, cur = 0, depth = 0;
  while (count > 0) {
    size_t need = (size_t)total + 2 * (size_t)count;
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
    launch_tree_level(first, count, nbegin.p, nend.p, leaf, bx[cur][0].p, bx[cur][1].p,
                      bx[cur][2].p, bx[cur][3].p, bp[cur].p, bx[nx][0].p, bx[nx][1].p,
                      bx[nx][2].p, bx[nx][3].p, bp[nx].p, box.p, nleft.p, s);
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
  op->n_leaves = (int)read1(scan.p + M, s);
  op->leaves.alloc(op->n_leaves);
  launch_leaf_list(M, flag.p, scan.p, start.p, op->leaves.p, s);
  op->leaf_of_node.alloc(total);
  fill_i32(op->leaf_of_node.p, -1, total, s);
  launch_leaf_index(op->n_leaves, op->leaves.p, op->leaf_of_node.p, s);
  HMX_HIP(hipStreamSynchronize(s));
  // the product holds one leaf's rows in a workgroup (at most 4 x 64); a leaf can exceed the
  // leaf size only when its points coincide
  std::vector<int32_t> hb, he, hc;
  to_host(hb, op->nbegin.p, total, s);
  to_host(he, op->nend.p, total, s);
  to_host(hc, op->child0.p, total, s);
  for (int i = 0; i < total; ++i)
    HMX_REQUIRE(hc[i] >= 0 || he[i] - hb[i] <= 256, HMX_EUNSUPPORTED,
                "a leaf holds more than 256 points (coincident points)");
}

// Sort a device list of (t, s) pairs into the lexicographic order of their node ranges.
void sort_pairs(hmx_op* op, DevBuf<int2>& L, int64_t n, hipStream_t s) {
  if (n <= 1) return;
  int64_t np = next_pow2(n);
  DevBuf<uint64_t> key(np);
  DevBuf<int32_t> val(np);
  launch_pair_keys(L.p, n, np, op->nbegin.p, op->nlevel.p, key.p, val.p, s);
  sort_u64_pairs(key.p, val.p, np, s);
  DevBuf<int2> out(n);
  launch_pair_gather(L.p, val.p, n, out.p, s);
  HMX_HIP(hipStreamSynchronize(s));
  L = std::move(out);
}

// ------------------------------------------------------------------------------ block tree
void build_blocks(hmx_op* op, hipStream_t s) {
  const double eta2 = op->p.eta * op->p.eta;
  size_t fcap = 1024, ncap = std::max<size_t>(1024, 64 * (size_t)op->n_leaves),
         xcap = std::max<size_t>(1024, 64 * (size_t)op->n_leaves);
  DevBuf<int2> front(fcap), next(fcap), nearL(ncap), farL(xcap);
  DevBuf<int> cnt(3);  // next, near, far
  fill_i32(cnt.p, 0, 3, s);
  int2 root = make_int2(0, 0);
  HMX_HIP(hipMemcpyAsync(front.p, &root, sizeof(int2), hipMemcpyHostToDevice, s));
  int64_t nfront = 1, n_near = 0, n_far = 0;
  while (nfront > 0) {
    if ((size_t)(4 * nfront) > next.n) {
      next.alloc(std::max<size_t>(4 * nfront, 2 * next.n));
    }
    if (nearL.n < (size_t)(n_near + nfront)) grow(nearL, 2 * (n_near + nfront), n_near, s);
    if (farL.n < (size_t)(n_far + nfront)) grow(farL, 2 * (n_far + nfront), n_far, s);
    fill_i32(cnt.p, 0, 1, s);
    launch_block_level(front.p, (int)nfront, op->box.p, op->child0.p, op->child1.p, eta2, next.p,
                       cnt.p, nearL.p, cnt.p + 1, farL.p, cnt.p + 2, s);
    int c[3];
    HMX_HIP(hipMemcpyAsync(c, cnt.p, sizeof(c), hipMemcpyDeviceToHost, s));
    HMX_HIP(hipStreamSynchronize(s));
    nfront = c[0];
    n_near = c[1];
    n_far = c[2];
    std::swap(front, next);
  }
  op->n_near = n_near;
  op->n_far = n_far;
  sort_pairs(op, nearL, n_near, s);
  sort_pairs(op, farL, n_far, s);
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
  size_t bytes = (size_t)op->near_entries * sizeof(T);
  if (op->p.pool_limit_bytes > 0 && (int64_t)bytes > op->p.pool_limit_bytes)
    throw Error(HMX_ENOMEM, "near field exceeds pool_limit_bytes");
  op->near_pool.alloc(std::max<size_t>(bytes, 1));
  launch_assemble<T>(op->near_tb.p, op->near_m.p, op->near_sb.p, op->near_n.p, op->near_off.p, nn,
                     op->X.p, op->Y.p, op->Z.p, op->W.p, op->kern, op->k, (T*)op->near_pool.p, s);
  HMX_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------ far field
template <class T>
void build_far(hmx_op* op, hipStream_t s) {
  const int64_t nf = op->n_far;
  const int nl = op->n_leaves;
  DevBuf<int32_t> ftb(std::max<int64_t>(nf, 1)), fm(std::max<int64_t>(nf, 1)),
      fsb(std::max<int64_t>(nf, 1)), fn(std::max<int64_t>(nf, 1));
  DevBuf<int64_t> node_cnt(op->n_nodes);
  DevBuf<int32_t> node_first(op->n_nodes);
  fill_i64(node_cnt.p, 0, op->n_nodes, s);
  fill_i32(node_first.p, -1, op->n_nodes, s);
  launch_far_prep(op->farL.p, nf, op->nbegin.p, op->nend.p, ftb.p, fm.p, fsb.p, fn.p, node_cnt.p,
                  node_first.p, s);
  std::vector<int32_t> htb, hm, hsb, hn;
  to_host(htb, ftb.p, nf, s);
  to_host(hm, fm.p, nf, s);
  to_host(hsb, fsb.p, nf, s);
  to_host(hn, fn.p, nf, s);

  // first slots
  std::vector<FarDesc> desc(nf);
  int64_t pool_elems = 0, flag_bytes = 0;
  for (int64_t b = 0; b < nf; ++b) {
    FarDesc& d = desc[b];
    d.tb = htb[b];
    d.m = hm[b];
    d.sb = hsb[b];
    d.n = hn[b];
    int64_t rc = ((int64_t)d.m * d.n) / ((int64_t)d.m + d.n);
    rc = std::min<int64_t>(rc, ACA_COEF_MAX);
    if (op->p.force_rank_cap > 0) rc = std::min<int64_t>(rc, op->p.force_rank_cap);
    d.rcap = (int32_t)rc;
    d.cap = (int32_t)std::min<int64_t>(rc, op->p.initial_rank);
    pool_elems += (int64_t)d.cap * (d.m + d.n);
    d.foff = flag_bytes;
    flag_bytes += d.m + d.n;
  }
  std::vector<DevBuf<T>> pools;
  pools.emplace_back(std::max<int64_t>(pool_elems, 1));
  {
    T* base = pools.back().p;
    int64_t off = 0;
    for (auto& d : desc) {
      d.U = base + off;
      off += (int64_t)d.cap * d.m;
      d.V = base + off;
      off += (int64_t)d.cap * d.n;
    }
  }
  DevBuf<uint8_t> flags(std::max<int64_t>(flag_bytes, 1));
  // largest blocks first
  std::vector<int32_t> order(nf);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return (int64_t)desc[a].m + desc[a].n > (int64_t)desc[b].m + desc[b].n;
  });
  DevBuf<FarDesc> d_desc(std::max<int64_t>(nf, 1));
  DevBuf<int32_t> d_order(std::max<int64_t>(nf, 1)), rank(std::max<int64_t>(nf, 1)),
      ipiv(std::max<int64_t>(nf, 1)), status(std::max<int64_t>(nf, 1));
  DevBuf<double> norm2(std::max<int64_t>(nf, 1));
  DevBuf<int> counter(1);
  if (nf) {
    HMX_HIP(hipMemcpyAsync(d_desc.p, desc.data(), nf * sizeof(FarDesc), hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(d_order.p, order.data(), nf * 4, hipMemcpyHostToDevice, s));
  }
  fill_i32(counter.p, 0, 1, s);
  launch_aca<T>(d_desc.p, d_order.p, (int)nf, counter.p, op->X.p, op->Y.p, op->Z.p, op->W.p,
                op->kern, op->k, op->p.tol, flags.p, rank.p, ipiv.p, status.p, norm2.p, 1, s);
  std::vector<int32_t> hst, hrank;
  to_host(hst, status.p, nf, s);
  // continue blocks that outgrew their slot in larger slots
  int64_t overflowed = 0;
  for (;;) {
    std::vector<int32_t> list;
    for (int64_t b = 0; b < nf; ++b)
      if (hst[b] == ACA_OVERFLOW) list.push_back((int32_t)b);
    if (list.empty()) break;
    overflowed += (int64_t)list.size();
    to_host(hrank, rank.p, nf, s);
    std::vector<FarDesc> nd = desc;
    int64_t extra = 0;
    for (int32_t b : list) {
      FarDesc& d = nd[b];
      d.cap = (int32_t)std::min<int64_t>(d.rcap, std::max<int64_t>(2 * (int64_t)d.cap, d.cap + 8));
      extra += (int64_t)d.cap * (d.m + d.n);
    }
    pools.emplace_back(extra);
    T* base = pools.back().p;
    int64_t off = 0;
    for (int32_t b : list) {
      FarDesc& d = nd[b];
      d.U = base + off;
      off += (int64_t)d.cap * d.m;
      d.V = base + off;
      off += (int64_t)d.cap * d.n;
    }
    DevBuf<FarDesc> d_nd(nf);
    DevBuf<int32_t> d_list(list.size());
    HMX_HIP(hipMemcpyAsync(d_nd.p, nd.data(), nf * sizeof(FarDesc), hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(d_list.p, list.data(), list.size() * 4, hipMemcpyHostToDevice, s));
    launch_copy_factors<T>(d_desc.p, d_nd.p, rank.p, d_list.p, (int)list.size(), s);
    HMX_HIP(hipStreamSynchronize(s));
    desc.swap(nd);
    d_desc = std::move(d_nd);
    fill_i32(counter.p, 0, 1, s);
    launch_aca<T>(d_desc.p, d_list.p, (int)list.size(), counter.p, op->X.p, op->Y.p, op->Z.p,
                  op->W.p, op->kern, op->k, op->p.tol, flags.p, rank.p, ipiv.p, status.p, norm2.p,
                  0, s);
    to_host(hst, status.p, nf, s);
  }
  op->overflow_blocks = overflowed;
  to_host(hrank, rank.p, nf, s);

  // final layout: U (m x r) then V (n x r) per block; dense blocks hold K (m x n)
  std::vector<FarRec> rec(nf);
  int64_t run = 0, trun = 0;
  std::vector<int32_t> dtb, dm, dsb, dn;
  std::vector<int64_t> doff;
  op->far_entries = op->dense_far = op->dense_far_entries = op->max_rank = op->sum_rank = 0;
  int64_t evals = 0;
  for (int64_t b = 0; b < nf; ++b) {
    const FarDesc& d = desc[b];
    FarRec& f = rec[b];
    f.tb = d.tb;
    f.m = d.m;
    f.sb = d.sb;
    f.n = d.n;
    HMX_REQUIRE(hst[b] == ACA_CONVERGED || hst[b] == ACA_DENSE, HMX_EINTERNAL,
                "ACA left a block unfinished");
    if (hst[b] == ACA_DENSE) {
      f.dense = 1;
      f.r = d.n;
      f.uoff = run;
      f.voff = run;
      run += (int64_t)d.m * d.n;
      f.toff = trun;
      trun += d.n;
      op->dense_far++;
      op->dense_far_entries += (int64_t)d.m * d.n;
      dtb.push_back(d.tb);
      dm.push_back(d.m);
      dsb.push_back(d.sb);
      dn.push_back(d.n);
      doff.push_back(f.uoff);
      evals += (int64_t)d.m * d.n + (int64_t)hrank[b] * (d.m + d.n);
    } else {
      f.dense = 0;
      f.r = hrank[b];
      f.uoff = run;
      run += (int64_t)f.r * d.m;
      f.voff = run;
      run += (int64_t)f.r * d.n;
      f.toff = trun;
      trun += f.r;
      op->far_entries += (int64_t)f.r * (d.m + d.n);
      op->max_rank = std::max<int64_t>(op->max_rank, f.r);
      op->sum_rank += f.r;
      evals += (int64_t)f.r * (d.m + d.n);
    }
  }
  op->kernel_evals += evals;
  size_t bytes = (size_t)run * sizeof(T);
  if (op->p.pool_limit_bytes > 0 &&
      (int64_t)(bytes + op->near_pool.bytes()) > op->p.pool_limit_bytes)
    throw Error(HMX_ENOMEM, "operator exceeds pool_limit_bytes");
  op->far_pool.alloc(std::max<size_t>(bytes, 1));
  op->far_pool_elems = run;
  op->t_len = trun;
  op->far.alloc(std::max<int64_t>(nf, 1));
  if (nf) HMX_HIP(hipMemcpyAsync(op->far.p, rec.data(), nf * sizeof(FarRec), hipMemcpyHostToDevice, s));
  launch_compact<T>(d_desc.p, op->far.p, rank.p, nf, (T*)op->far_pool.p, s);
  if (!dtb.empty()) {
    int64_t nd = (int64_t)dtb.size();
    DevBuf<int32_t> a(nd), b2(nd), c(nd), e(nd);
    DevBuf<int64_t> o(nd);
    HMX_HIP(hipMemcpyAsync(a.p, dtb.data(), nd * 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(b2.p, dm.data(), nd * 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(c.p, dsb.data(), nd * 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(e.p, dn.data(), nd * 4, hipMemcpyHostToDevice, s));
    HMX_HIP(hipMemcpyAsync(o.p, doff.data(), nd * 8, hipMemcpyHostToDevice, s));
    launch_assemble<T>(a.p, b2.p, c.p, e.p, o.p, nd, op->X.p, op->Y.p, op->Z.p, op->W.p, op->kern,
                       op->k, (T*)op->far_pool.p, s);
    HMX_HIP(hipStreamSynchronize(s));
  }
  HMX_HIP(hipStreamSynchronize(s));
  op->far_host = std::move(rec);

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
  op->kernel_evals += op->near_entries;
  op->t_near = tm.stop();
  build_far<T>(op, s);
  op->t_aca = tm.stop();
  op->xp.alloc((size_t)op->M * sizeof(T));
  op->tbuf.alloc(std::max<size_t>((size_t)op->t_len * sizeof(T), sizeof(T)));
  op->t_total = total.stop();
}

void finish_build(hmx_op* op, hipStream_t s) {
  const size_t es = op->prec == HMX_FP64 ? sizeof(double2) : sizeof(float2);
  op->elem = es;
  if (op->p.tol <= 0) {
    op->dense = true;
    op->partial.alloc((size_t)dense_otf_partial_len(op->M) * es);
    return;
  }
  if (op->prec == HMX_FP64) build_h<double2>(op, s);
  else build_h<float2>(op, s);
}

void check_build_args(int32_t kern, double k) {
  HMX_REQUIRE(kern == HMX_LAPLACE || kern == HMX_HELMHOLTZ || kern == HMX_TEST_POLY2, HMX_EINVAL,
              "unknown kernel");
  HMX_REQUIRE(std::isfinite(k) && k >= 0, HMX_EINVAL, "k must be finite and >= 0");
}

}  // namespace

int64_t hmx_op::bytes() const {
  size_t b = X.bytes() + Y.bytes() + Z.bytes() + W.bytes() + perm.bytes() + nbegin.bytes() +
             nend.bytes() + nlevel.bytes() + child0.bytes() + child1.bytes() + parent.bytes() +
             box.bytes() + leaves.bytes() + leaf_of_node.bytes() + nearL.bytes() + near_tb.bytes() +
             near_m.bytes() + near_sb.bytes() + near_n.bytes() + near_off.bytes() +
             near_ptr.bytes() + near_pool.bytes() + farL.bytes() + far.bytes() + far_pool.bytes() +
             far_ptr.bytes() + far_list.bytes() + xp.bytes() + tbuf.bytes() + partial.bytes();
  return (int64_t)b;
}

extern "C" {

hmx_status hmx_params_default(hmx_params* p) {
  if (!p) return fail(HMX_EINVAL, "null params");
  defaults(p);
  return HMX_OK;
}

hmx_status hmx_quad_points(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                           const double* q_bary, const double* q_w, int32_t n_q, double* xyzw,
                           void* stream) {
  API_TRY
  HMX_REQUIRE(vtx && tri && xyzw, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 1 && n_tri >= 1, HMX_EINVAL, "empty mesh");
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  const int64_t M = n_tri * n_q;
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, xyzw, xyzw + M, xyzw + 2 * M, xyzw + 3 * M, err.p, s);
  int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_build(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                     const double* q_bary, const double* q_w, int32_t n_q, int32_t kern, double k,
                     const hmx_params* p, void* stream, hmx_op** out) {
  API_TRY
  HMX_REQUIRE(vtx && tri && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 1 && n_tri >= 1, HMX_EINVAL, "empty mesh");
  check_build_args(kern, k);
  hmx_params prm = resolve(p);
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  auto op = std::make_unique<hmx_op>();
  op->M = n_tri * n_q;
  op->kern = kern;
  op->k = k;
  op->p = prm;
  op->prec = prm.precision;
  op->X.alloc(op->M);
  op->Y.alloc(op->M);
  op->Z.alloc(op->M);
  op->W.alloc(op->M);
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, op->X.p, op->Y.p, op->Z.p, op->W.p, err.p, s);
  int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_build_points(const double* xyzw, int64_t M, int32_t kern, double k,
                            const hmx_params* p, void* stream, hmx_op** out) {
  API_TRY
  HMX_REQUIRE(xyzw && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(M >= 1, HMX_EINVAL, "M must be >= 1");
  check_build_args(kern, k);
  hmx_params prm = resolve(p);
  hipStream_t s = as_stream(stream);
  auto op = std::make_unique<hmx_op>();
  op->M = M;
  op->kern = kern;
  op->k = k;
  op->p = prm;
  op->prec = prm.precision;
  op->X.alloc(M);
  op->Y.alloc(M);
  op->Z.alloc(M);
  op->W.alloc(M);
  HMX_HIP(hipMemcpyAsync(op->X.p, xyzw, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->Y.p, xyzw + M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->Z.p, xyzw + 2 * M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->W.p, xyzw + 3 * M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipStreamSynchronize(s));
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_matvec(const hmx_op* op, const void* x, void* y, void* stream) {
  API_TRY
  HMX_REQUIRE(op && x && y, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(x != y, HMX_EINVAL, "x and y must not alias");
  hipStream_t s = as_stream(stream);
  if (op->dense) {
    if (op->prec == HMX_FP64)
      launch_dense_otf<double2>(op->X.p, op->Y.p, op->Z.p, op->W.p, op->M, op->kern, op->k,
                                (const double2*)x, (double2*)op->partial.p, (double2*)y, s);
    else
      launch_dense_otf<float2>(op->X.p, op->Y.p, op->Z.p, op->W.p, op->M, op->kern, op->k,
                               (const float2*)x, (float2*)op->partial.p, (float2*)y, s);
    return HMX_OK;
  }
  auto run = [&](auto tag) {
    using T = decltype(tag);
    T* xp = (T*)op->xp.p;
    T* t = (T*)op->tbuf.p;
    launch_gather<T>((const T*)x, op->perm.p, xp, op->M, s);
    launch_far_vt<T>(op->far.p, op->n_far, (const T*)op->far_pool.p, xp, t, s);
    launch_leaf_apply<T>(op->n_leaves, op->leaves.p, op->nbegin.p, op->nend.p, op->near_ptr.p,
                         op->near_sb.p, op->near_n.p, op->near_off.p, (const T*)op->near_pool.p,
                         op->far_ptr.p, op->far_list.p, op->far.p, (const T*)op->far_pool.p, t, xp,
                         op->perm.p, (T*)y, s);
  };
  if (op->prec == HMX_FP64) run(double2{});
  else run(float2{});
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_info(const hmx_op* op, hmx_info_t* out) {
  if (!op || !out) return fail(HMX_EINVAL, "null pointer");
  std::memset(out, 0, sizeof(*out));
  out->n_points = op->M;
  out->n_nodes = op->n_nodes;
  out->n_leaves = op->n_leaves;
  out->n_near = op->n_near;
  out->n_far = op->n_far;
  out->near_entries = op->near_entries;
  out->far_entries = op->far_entries;
  out->dense_far = op->dense_far;
  out->dense_far_entries = op->dense_far_entries;
  out->max_rank = op->max_rank;
  out->sum_rank = op->sum_rank;
  out->overflow_blocks = op->overflow_blocks;
  out->bytes = op->bytes();
  out->precision = op->prec;
  out->is_dense = op->dense ? 1 : 0;
  out->t_tree_ms = op->t_tree;
  out->t_blocks_ms = op->t_blocks;
  out->t_near_ms = op->t_near;
  out->t_aca_ms = op->t_aca;
  out->t_total_ms = op->t_total;
  out->kernel_evals = op->kernel_evals;
  return HMX_OK;
}

hmx_status hmx_export_tree(const hmx_op* op, int32_t* perm, int64_t* begin, int64_t* end,
                           int32_t* level, int32_t* child0, int32_t* child1, double* box) {
  API_TRY
  HMX_REQUIRE(op, HMX_EINVAL, "null operator");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no tree");
  hipStream_t s = nullptr;
  const int n = op->n_nodes;
  std::vector<int32_t> tmp;
  if (perm) {
    to_host(tmp, op->perm.p, op->M, s);
    std::memcpy(perm, tmp.data(), op->M * 4);
  }
  if (begin) {
    to_host(tmp, op->nbegin.p, n, s);
    for (int i = 0; i < n; ++i) begin[i] = tmp[i];
  }
  if (end) {
    to_host(tmp, op->nend.p, n, s);
    for (int i = 0; i < n; ++i) end[i] = tmp[i];
  }
  if (level) {
    to_host(tmp, op->nlevel.p, n, s);
    std::memcpy(level, tmp.data(), n * 4);
  }
  if (child0) {
    to_host(tmp, op->child0.p, n, s);
    std::memcpy(child0, tmp.data(), n * 4);
  }
  if (child1) {
    to_host(tmp, op->child1.p, n, s);
    std::memcpy(child1, tmp.data(), n * 4);
  }
  if (box) {
    std::vector<double> hb;
    to_host(hb, op->box.p, 6 * (size_t)n, s);
    std::memcpy(box, hb.data(), 6 * (size_t)n * 8);
  }
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_export_blocks(const hmx_op* op, int64_t* near_rc, int64_t* far_rc, int32_t* ranks) {
  API_TRY
  HMX_REQUIRE(op, HMX_EINVAL, "null operator");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no blocks");
  hipStream_t s = nullptr;
  if (near_rc && op->n_near) {
    std::vector<int32_t> a, b, c, d;
    to_host(a, op->near_tb.p, op->n_near, s);
    to_host(b, op->near_m.p, op->n_near, s);
    to_host(c, op->near_sb.p, op->n_near, s);
    to_host(d, op->near_n.p, op->n_near, s);
    for (int64_t i = 0; i < op->n_near; ++i) {
      near_rc[4 * i] = a[i];
      near_rc[4 * i + 1] = a[i] + b[i];
      near_rc[4 * i + 2] = c[i];
      near_rc[4 * i + 3] = c[i] + d[i];
    }
  }
  for (int64_t i = 0; i < op->n_far; ++i) {
    const FarRec& f = op->far_host[i];
    if (far_rc) {
      far_rc[4 * i] = f.tb;
      far_rc[4 * i + 1] = f.tb + f.m;
      far_rc[4 * i + 2] = f.sb;
      far_rc[4 * i + 3] = f.sb + f.n;
    }
    if (ranks) ranks[i] = f.dense ? -1 : f.r;
  }
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_export_far(const hmx_op* op, int64_t b, void* U, void* V, int32_t* rank) {
  API_TRY
  HMX_REQUIRE(op && U && rank, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no far blocks");
  HMX_REQUIRE(b >= 0 && b < op->n_far, HMX_EINVAL, "far block index out of range");
  const FarRec& f = op->far_host[b];
  const char* base = (const char*)op->far_pool.p;
  if (f.dense) {
    HMX_HIP(hipMemcpy(U, base + f.uoff * op->elem, (size_t)f.m * f.n * op->elem, hipMemcpyDeviceToHost));
    *rank = -1;
  } else {
    HMX_REQUIRE(V || f.r == 0, HMX_EINVAL, "null V");
    if (f.r) {
      HMX_HIP(hipMemcpy(U, base + f.uoff * op->elem, (size_t)f.m * f.r * op->elem, hipMemcpyDeviceToHost));
      HMX_HIP(hipMemcpy(V, base + f.voff * op->elem, (size_t)f.n * f.r * op->elem, hipMemcpyDeviceToHost));
    }
    *rank = f.r;
  }
  return HMX_OK;
  API_CATCH
}

void hmx_destroy(hmx_op* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  delete op;
}

const char* hmx_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// k_far.hip -- device-side bookkeeping of the far field around ACA: block descriptors (rank cap,
// first slot size, used-flag offsets, pool estimate), the class / size ordering of the ACA
// launch, and after ACA the product's block records, the statistics and the list of blocks
// stored dense.  None of this is arithmetic of the method; it replaces host loops over all far
// blocks and the transfers they need.
#include <limits.h>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

// Descriptor of far block b (pair (t, s) of tree nodes): rows [tb, tb + m), columns [sb, sb + n),
// rank cap min(floor(mn / (m + n)), ACA_COEF_MAX, force_cap), first slot of initial_rank columns
// (twice / three times that for m + n >= ACA_BIG / 2 ACA_BIG), no slot yet; wavefront class
// (m, n <= ACA_WAVE_N) only when use_wave.
__global__ void __launch_bounds__(WG) far_desc_kernel(
    const int2* __restrict__ pairs, int64_t nf, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, int initial_rank, int force_cap, int use_wave,
    FarDesc* __restrict__ desc,
    int64_t* __restrict__ mn_out, int64_t* __restrict__ est, uint8_t* __restrict__ wave,
    int64_t* __restrict__ work) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (b >= nf) return;
  const int2 p = pairs[b];
  FarDesc d;
  d.tb = nbegin[p.x];
  d.m = nend[p.x] - d.tb;
  d.sb = nbegin[p.y];
  d.n = nend[p.y] - d.sb;
  const int64_t mn = (int64_t)d.m + d.n;
  int64_t rc = ((int64_t)d.m * d.n) / mn;
  rc = rc < ACA_COEF_MAX ? rc : ACA_COEF_MAX;
  if (force_cap > 0 && rc > force_cap) rc = force_cap;
  d.rcap = (int32_t)rc;
  const int64_t c0 = mn >= 2 * ACA_BIG ? 3 * (int64_t)initial_rank
                     : mn >= ACA_BIG   ? 2 * (int64_t)initial_rank
                                       : (int64_t)initial_rank;
  d.cap = (int32_t)(c0 < rc ? c0 : rc);
  d.U = nullptr;
  d.U1 = nullptr;
  d.foff = 0;
  d.ld = (int32_t)mn;
  d.cap1 = 0;
  desc[b] = d;
  const bool w = use_wave && d.m <= ACA_WAVE_N && d.n <= ACA_WAVE_N;
  wave[b] = w ? 1 : 0;
  mn_out[b] = mn;
  // pool estimate without a rank model (generous: a short pool costs another launch round):
  // wavefront blocks take exactly their rank (<= 16, typically ~8), workgroup blocks twice their
  // first slot size
  est[b] = w ? 12 * mn : 2 * (int64_t)d.cap * mn;
  work[b] = mn;
}

__global__ void __launch_bounds__(WG) far_foff_kernel(FarDesc* __restrict__ desc,
                                                      const int64_t* __restrict__ foff, int64_t nf) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (b < nf) desc[b].foff = foff[b];
}

// Learned model: r_alloc = min(rcap, ceil(alpha * max(expm1(pred) * scale, 0)) + beta), at least
// 1 when rcap > 0; r_alloc (m + n) entries and the work key r_alloc^2 (m + n).
__global__ void __launch_bounds__(WG) far_pred_kernel(const float* __restrict__ pred,
                                                      const FarDesc* __restrict__ desc,
                                                      int64_t nf, double alpha, int64_t beta,
                                                      double scale, int64_t* __restrict__ ramn,
                                                      int64_t* __restrict__ work) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (b >= nf) return;
  const FarDesc d = desc[b];
  const double rhat = expm1((double)pred[b]) * scale;
  int64_t ra = (int64_t)ceil(alpha * fmax(rhat, 0.0)) + beta;
  if (ra < (d.rcap > 0 ? 1 : 0)) ra = d.rcap > 0 ? 1 : 0;
  if (ra > d.rcap) ra = d.rcap;
  const int64_t mn = (int64_t)d.m + d.n, r1 = ra > 1 ? ra : 1;
  ramn[b] = ra * mn;
  work[b] = r1 * r1 * mn;
}

// ACA class of a block that has not started: 0 for m + n >= big_mn, 2 for wavefront blocks, 3
// for m + n < small_mn with rank cap <= ACA_COEF_SMALL, 1 otherwise.
__device__ __forceinline__ int far_class(const FarDesc& d, uint8_t wave, int64_t big_mn,
                                         int64_t small_mn) {
  const int64_t mn = (int64_t)d.m + d.n;
  return mn >= big_mn ? 0 : wave ? 2 : (mn < small_mn && d.rcap <= ACA_COEF_SMALL) ? 3 : 1;
}

// Launch order: key = class * 64 + (63 - floor(log2 work)); blocks are counted per key, the
// counts scanned, and each block placed in its key's range (order inside a key is arbitrary).
constexpr int ORDER_KEYS = FAR_ORDER_KEYS;

__device__ __forceinline__ int far_key(const FarDesc& d, uint8_t wave, int64_t work,
                                       int64_t big_mn, int64_t small_mn) {
  const int cls = far_class(d, wave, big_mn, small_mn);
  const int lw = 63 - __clzll((unsigned long long)(work > 1 ? work : 1));
  return cls * 64 + (63 - lw);
}

__global__ void __launch_bounds__(WG) far_key_hist_kernel(const FarDesc* __restrict__ desc,
                                                          const uint8_t* __restrict__ wave,
                                                          const int64_t* __restrict__ work,
                                                          int64_t nf, int64_t big_mn,
                                                          int64_t small_mn,
                                                          int* __restrict__ hist) {
  __shared__ int lh[ORDER_KEYS];
  for (int q = threadIdx.x; q < ORDER_KEYS; q += WG) lh[q] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (b < nf) atomicAdd(&lh[far_key(desc[b], wave[b], work[b], big_mn, small_mn)], 1);
  __syncthreads();
  for (int q = threadIdx.x; q < ORDER_KEYS; q += WG)
    if (lh[q]) atomicAdd(&hist[q], lh[q]);
}

// cursor[q] = sum_{q' < q} hist[q'] (one workgroup).
__global__ void __launch_bounds__(WG) far_key_scan_kernel(const int* __restrict__ hist,
                                                          int* __restrict__ cursor) {
  __shared__ int s[NWAVE];
  int run = 0;
  for (int c = 0; c < ORDER_KEYS; c += WG) {
    const int q = c + threadIdx.x;
    const int v = q < ORDER_KEYS ? hist[q] : 0;
    int tot;
    const int pre = block_excl_scan(v, s, &tot);
    if (q < ORDER_KEYS) cursor[q] = run + pre;
    run += tot;
  }
}

__global__ void __launch_bounds__(WG) far_key_scatter_kernel(const FarDesc* __restrict__ desc,
                                                             const uint8_t* __restrict__ wave,
                                                             const int64_t* __restrict__ work,
                                                             int64_t nf, int64_t big_mn,
                                                             int64_t small_mn,
                                                             int* __restrict__ cursor,
                                                             int32_t* __restrict__ order) {
  __shared__ int lh[ORDER_KEYS], base[ORDER_KEYS];
  for (int q = threadIdx.x; q < ORDER_KEYS; q += WG) lh[q] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  int key = 0, local = 0;
  if (b < nf) {
    key = far_key(desc[b], wave[b], work[b], big_mn, small_mn);
    local = atomicAdd(&lh[key], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ORDER_KEYS; q += WG)
    if (lh[q]) base[q] = atomicAdd(&cursor[q], lh[q]);
  __syncthreads();
  if (b < nf) order[base[key] + local] = (int32_t)b;
}

// Records of the product after ACA, with per-block counts for the offset scans:
// tcount = length of the block's t segment (r, or n for a dense block), dcount = m n for a dense
// block, dflag = 1 for a dense block; stats (int64 atomics): [0] far entries sum r (m + n),
// [1] sum of ranks, [2] max rank, [3] dense blocks, [4] dense entries, [5] blocks that moved to a
// larger slot or were continued in a later round, [6] kernel evaluations, [7 + c] blocks of
// first-launch class c, [11 + c] bytes ACA must move in class c: es (m + n) r (r + 1) / 2 per
// block (step k reads the k previous columns of U and V once and writes one column pair).
__global__ void __launch_bounds__(WG) far_rec_kernel(
    const FarDesc* __restrict__ desc, const int32_t* __restrict__ rank,
    const int32_t* __restrict__ status, const uint8_t* __restrict__ continued,
    const uint8_t* __restrict__ wave, int64_t big_mn, int64_t small_mn, int es, int64_t nf,
    FarRec* __restrict__ rec, int64_t* __restrict__ tcount, int64_t* __restrict__ dcount,
    int64_t* __restrict__ dflag, unsigned long long* __restrict__ stats, int* __restrict__ bad) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  unsigned long long v[FAR_STATS] = {};
  if (b < nf) {
    const FarDesc d = desc[b];
    const int32_t st = status[b] & 0xff;
    if (st != ACA_CONVERGED && st != ACA_DENSE) atomicOr(bad, 1);
    const bool dense = st == ACA_DENSE;
    const int64_t r = rank[b];
    FarRec f;
    f.tb = d.tb;
    f.m = d.m;
    f.sb = d.sb;
    f.n = d.n;
    f.dense = dense ? 1 : 0;
    f.r = dense ? d.n : (int32_t)r;
    // factors: interleaved column pairs in up to two segments (V = U + m within a segment)
    const size_t es_m = (size_t)es * d.m;
    f.U = dense ? nullptr : d.U;
    f.V = dense || !d.U ? nullptr : (const void*)((const char*)d.U + es_m);
    f.toff = 0;
    f.ldu = dense ? d.m : d.ld;
    f.ldv = dense ? d.n : d.ld;
    f.split = dense ? d.n : d.cap;
    f.pad_ = 0;
    f.U1 = dense ? nullptr : d.U1;
    f.V1 = dense || !d.U1 ? nullptr : (const void*)((const char*)d.U1 + es_m);
    rec[b] = f;
    const int64_t mn = (int64_t)d.m + d.n, mxn = (int64_t)d.m * d.n;
    tcount[b] = dense ? d.n : r;
    dcount[b] = dense ? mxn : 0;
    dflag[b] = dense ? 1 : 0;
    if (!dense) {
      v[0] = r * mn;
      v[1] = r;
      v[2] = r;
    } else {
      v[3] = 1;
      v[4] = mxn;
    }
    v[5] = ((status[b] & ACA_GREW) || (continued && continued[b])) ? 1 : 0;
    v[6] = dense ? mxn + r * mn : r * mn;
    const int cls = far_class(d, wave[b], big_mn, small_mn);
    v[7 + cls] = 1;
    v[11 + cls] = (int64_t)es * mn * r * (r + 1) / 2;
  }
  // one atomic per workgroup and statistic (wavefront sums, then the four wavefronts in LDS):
  // one per wavefront kept thousands of atomics queued on each of the few addresses
  __shared__ unsigned long long wsum[NWAVE][FAR_STATS];
  const int lane = threadIdx.x & 63, w = threadIdx.x / WAVE;
#pragma unroll
  for (int q = 0; q < FAR_STATS; ++q) {
    unsigned long long x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(x, o, 64);
      x = q == 2 ? (x > y ? x : y) : x + y;
    }
    if (lane == 0) wsum[w][q] = x;
  }
  __syncthreads();
  if (threadIdx.x < FAR_STATS) {
    const int q = threadIdx.x;
    unsigned long long x = wsum[0][q];
#pragma unroll
    for (int u = 1; u < NWAVE; ++u) x = q == 2 ? (x > wsum[u][q] ? x : wsum[u][q]) : x + wsum[u][q];
    if (x) {
      if (q == 2)
        atomicMax(&stats[q], x);
      else
        atomicAdd(&stats[q], x);
    }
  }
}

// t offsets, dense slots, and the compact list of dense blocks for their assembly.
template <class T>
__global__ void __launch_bounds__(WG) far_rec_finish_kernel(
    FarRec* __restrict__ rec, const int64_t* __restrict__ toff, const int64_t* __restrict__ doff,
    const int64_t* __restrict__ dpos, int64_t nf, T* __restrict__ dense_pool,
    int32_t* __restrict__ dtb, int32_t* __restrict__ dm, int32_t* __restrict__ dsb,
    int32_t* __restrict__ dn, int64_t* __restrict__ dofs) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (b >= nf) return;
  FarRec f = rec[b];
  f.toff = toff[b];
  if (f.dense) {
    f.U = dense_pool + doff[b];
    const int64_t q = dpos[b];
    dtb[q] = f.tb;
    dm[q] = f.m;
    dsb[q] = f.sb;
    dn[q] = f.n;
    dofs[q] = doff[b];
  }
  rec[b] = f;
}

// Number of blocks whose status code (low byte) equals `code` (count starts at zero).
__global__ void __launch_bounds__(WG) far_count_status_kernel(const int32_t* __restrict__ status,
                                                              int64_t nf, int code,
                                                              int* __restrict__ count) {
  const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool hit = b < nf && (status[b] & 0xff) == code;
  const unsigned long long mask = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && mask) atomicAdd(count, (int)__popcll(mask));
}

// ------------------------------------------------------------------------------ launchers
static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + WG - 1) / WG)); }

void launch_far_desc(const int2* pairs, int64_t nf, const int32_t* nbegin, const int32_t* nend,
                     int initial_rank, int force_cap, int use_wave, FarDesc* desc, int64_t* mn, int64_t* est,
                     uint8_t* wave, int64_t* work, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_desc_kernel, grid_of(nf), dim3(WG), 0, s, pairs, nf, nbegin, nend,
                     initial_rank, force_cap, use_wave, desc, mn, est, wave, work);
  HMX_LAUNCHED();
}

void launch_far_foff(FarDesc* desc, const int64_t* foff, int64_t nf, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_foff_kernel, grid_of(nf), dim3(WG), 0, s, desc, foff, nf);
  HMX_LAUNCHED();
}

void launch_far_pred(const float* pred, const FarDesc* desc, int64_t nf, double alpha,
                     int64_t beta, double scale, int64_t* ramn, int64_t* work, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_pred_kernel, grid_of(nf), dim3(WG), 0, s, pred, desc, nf, alpha, beta,
                     scale, ramn, work);
  HMX_LAUNCHED();
}

void launch_far_order(const FarDesc* desc, const uint8_t* wave, const int64_t* work, int64_t nf,
                      int64_t big_mn, int64_t small_mn, int* hist, int* cursor, int32_t* order,
                      hipStream_t s) {
  if (nf <= 0) return;
  fill_i32(hist, 0, ORDER_KEYS, s);
  hipLaunchKernelGGL(far_key_hist_kernel, grid_of(nf), dim3(WG), 0, s, desc, wave, work, nf,
                     big_mn, small_mn, hist);
  hipLaunchKernelGGL(far_key_scan_kernel, dim3(1), dim3(WG), 0, s, hist, cursor);
  hipLaunchKernelGGL(far_key_scatter_kernel, grid_of(nf), dim3(WG), 0, s, desc, wave, work, nf,
                     big_mn, small_mn, cursor, order);
  HMX_LAUNCHED();
}

void launch_count_status(const int32_t* status, int64_t nf, int code, int* count, hipStream_t s) {
  fill_i32(count, 0, 1, s);
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_count_status_kernel, grid_of(nf), dim3(WG), 0, s, status, nf, code, count);
  HMX_LAUNCHED();
}

void launch_far_rec(const FarDesc* desc, const int32_t* rank, const int32_t* status,
                    const uint8_t* continued, const uint8_t* wave, int64_t big_mn,
                    int64_t small_mn, int es,
                    int64_t nf, FarRec* rec, int64_t* tcount, int64_t* dcount, int64_t* dflag,
                    unsigned long long* stats, int* bad, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_rec_kernel, grid_of(nf), dim3(WG), 0, s, desc, rank, status, continued,
                     wave, big_mn, small_mn, es, nf, rec, tcount, dcount, dflag, stats, bad);
  HMX_LAUNCHED();
}

template <class T>
void launch_far_rec_finish(FarRec* rec, const int64_t* toff, const int64_t* doff,
                           const int64_t* dpos, int64_t nf, T* dense_pool, int32_t* dtb,
                           int32_t* dm, int32_t* dsb, int32_t* dn, int64_t* dofs, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_rec_finish_kernel<T>, grid_of(nf), dim3(WG), 0, s, rec, toff, doff, dpos,
                     nf, dense_pool, dtb, dm, dsb, dn, dofs);
  HMX_LAUNCHED();
}

template void launch_far_rec_finish<double2>(FarRec*, const int64_t*, const int64_t*,
                                             const int64_t*, int64_t, double2*, int32_t*,
                                             int32_t*, int32_t*, int32_t*, int64_t*, hipStream_t);
template void launch_far_rec_finish<float2>(FarRec*, const int64_t*, const int64_t*,
                                            const int64_t*, int64_t, float2*, int32_t*, int32_t*,
                                            int32_t*, int32_t*, int64_t*, hipStream_t);

}  // namespace hmx

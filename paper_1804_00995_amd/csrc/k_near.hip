// k_near.hip -- assembly of dense blocks K_b[i, j] = G(x_{t+i}, x_{s+j}) w_{s+j}, column-major
// (element (i, j) at j * m + i), used for the near field and for far blocks stored dense.  With
// the singular correction (Section 5.2) the near-field kernel also corrects its block's close
// pairs, in place, right after assembling it.
#include "hmx_dev.h"
#include "hmx_host.h"
#include "hmx_reg_dev.h"

namespace hmx {

// One workgroup per block, in one of two layouts chosen per precision (measured):
//  - FP64 (an evaluation is about 100 VALU instructions): consecutive threads take consecutive
//    entries of the column-major block, so every lane is busy whatever m is; thread e handles
//    entries e, e + WG, ... with (i, j) advanced incrementally (no per-entry division);
//  - FP32 mixed (about 40, so that the loads weigh more): each wavefront takes whole columns j
//    (uniform across its lanes, so the source point comes through scalar loads) and its lanes
//    the rows of a chunk of 64, whose targets are loaded once; lanes past the last row evaluate
//    a clamped row and store nothing.
template <class T>
__global__ void __launch_bounds__(WG) assemble_kernel(
    const int32_t* __restrict__ tb, const int32_t* __restrict__ mm, const int32_t* __restrict__ sb,
    const int32_t* __restrict__ nn, const int64_t* __restrict__ off, const double* __restrict__ X,
    const double* __restrict__ Y, const double* __restrict__ Z, const double* __restrict__ W,
    int kern, const double* __restrict__ kp, T* __restrict__ pool) {
  const int blk = blockIdx.x;
  const int t0 = tb[blk], m = mm[blk], s0 = sb[blk], n = nn[blk];
  const double k = kp[t0];  // wavenumber of the block's mesh
  T* K = pool + off[blk];
  if constexpr (sizeof(T) == 16) {
    const int64_t total = (int64_t)m * n;
    int i = threadIdx.x % m, j = threadIdx.x / m;
    const int di = WG % m, dj = WG / m;
    for (int64_t e = threadIdx.x; e < total; e += WG) {
      K[e] = eval_entry<T>(kern, k, X[t0 + i], Y[t0 + i], Z[t0 + i], X[s0 + j], Y[s0 + j],
                           Z[s0 + j], W[s0 + j]);
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        j += 1;
      }
    }
  } else {
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    for (int r0 = 0; r0 < m; r0 += WAVE) {
      const int i = min(r0 + lane, m - 1);
      const bool live = r0 + lane < m;
      const double tx = X[t0 + i], ty = Y[t0 + i], tz = Z[t0 + i];
      for (int j = w; j < n; j += NWAVE) {
        const T v = eval_entry<T>(kern, k, tx, ty, tz, X[s0 + j], Y[s0 + j], Z[s0 + j], W[s0 + j]);
        if (live) K[(int64_t)j * m + r0 + lane] = v;
      }
    }
  }
}

// Near blocks with the singular correction (one workgroup per block): the block is assembled as
// above, then its close pairs are corrected in place while its lines are still in L2.  A close
// pair's correction needs one y-integral over the source triangle, which serves the target with
// all three of the triangle's points, so the work is organised per (target, triangle): a
// triangle belongs to the first of its points among the block's columns.  The block's targets
// and its owned triangles' closeness data are staged in LDS (near blocks pair leaves, which hold
// at most REG_LEAF points); then the (target, owned triangle) pairs are scanned in chunks of
// REG_CHUNK: (1) closeness is tested from LDS and the close pairs are queued; (2) the queued
// integrals are computed with all lanes busy (FP64, the expensive part) and each of the
// triangle's points in the block gets its entry corrected.  Every corrected entry is written by
// exactly one thread.  Registers are allocated for four waves per SIMD (a few spilled: measured
// slightly faster than the unconstrained three; five spill too much).
constexpr int REG_CHUNK = 8 * WG;
constexpr int REG_LEAF = 256;

template <class T>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) assemble_reg_kernel(
    const int32_t* __restrict__ tb, const int32_t* __restrict__ mm, const int32_t* __restrict__ sb,
    const int32_t* __restrict__ nn, const int64_t* __restrict__ off, const double* __restrict__ X,
    const double* __restrict__ Y, const double* __restrict__ Z, const double* __restrict__ W,
    int kern, const double* __restrict__ kp, T* __restrict__ pool, RegArgs ra) {
  __shared__ double tgt[3][REG_LEAF];     // target coordinates
  __shared__ double cen[4][REG_LEAF];     // owned triangles: centroid, (alpha d_T)^2
  __shared__ int tri_of[REG_LEAF];        // owned triangles: index
  __shared__ int queue[REG_CHUNK];        // close pairs of the chunk: i + m * (owned slot)
  __shared__ int qn, no;
  const int blk = blockIdx.x;
  const int t0 = tb[blk], m = mm[blk], s0 = sb[blk], n = nn[blk];
  T* K = pool + off[blk];
  {
    const double k = kp[t0];
    int i = threadIdx.x % m, j = threadIdx.x / m;
    const int di = WG % m, dj = WG / m;
    for (int e = threadIdx.x; e < m * n; e += WG) {
      K[e] = eval_entry<T>(kern, k, X[t0 + i], Y[t0 + i], Z[t0 + i], X[s0 + j], Y[s0 + j],
                           Z[s0 + j], W[s0 + j]);
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        j += 1;
      }
    }
  }
  // (the barriers below also make the block's entries visible to every thread of the workgroup)
  if (threadIdx.x == 0) no = 0;
  for (int i = threadIdx.x; i < m; i += WG) {
    tgt[0][i] = X[t0 + i];
    tgt[1][i] = Y[t0 + i];
    tgt[2][i] = Z[t0 + i];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += WG) {
    const int32_t t = ra.perm[s0 + j] / 3;
    bool own = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int p = ra.iperm[3 * t + q] - s0;
      own = own && !(p >= 0 && p < j);
    }
    if (own) {
      const int k = atomicAdd(&no, 1);
      const double* g = ra.tgeo + (int64_t)t * TGEO;
      tri_of[k] = t;
#pragma unroll
      for (int c = 0; c < 4; ++c) cen[c][k] = g[9 + c];
    }
  }
  __syncthreads();
  const int total = m * no;
  for (int c0 = 0; c0 < total; c0 += REG_CHUNK) {
    const int ce = min(REG_CHUNK, total - c0);
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    for (int le = threadIdx.x; le < ce; le += WG) {
      const int e = c0 + le, k = e / m, i = e - k * m;
      // closeness in the written order without contraction, as the records were built
      const double cx = tgt[0][i] - cen[0][k], cy = tgt[1][i] - cen[1][k], cz = tgt[2][i] - cen[2][k];
      const double c2 = __dadd_rn(__dadd_rn(__dmul_rn(cx, cx), __dmul_rn(cy, cy)), __dmul_rn(cz, cz));
      if (c2 <= cen[3][k]) queue[atomicAdd(&qn, 1)] = e;
    }
    __syncthreads();
    const int nq = qn;
    for (int qi = threadIdx.x; qi < nq; qi += WG) {
      const int e = queue[qi], k = e / m, i = e - k * m;
      const int32_t t = tri_of[k];
      const double tx = tgt[0][i], ty = tgt[1][i], tz = tgt[2][i];
      double J[3];
      tri_lagrange3(ra.tgeo + (int64_t)t * TGEO, ra.lag, tx, ty, tz, J);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int p = ra.iperm[3 * t + q] - s0;  // column of the triangle's point q
        if (p < 0 || p >= n) continue;
        const double dx = tx - X[s0 + p], dy = ty - Y[s0 + p], dz = tz - Z[s0 + p];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double gauss = r2 == 0.0 ? 0.0 : W[s0 + p] / sqrt(r2);
        T* ep = K + (int64_t)p * m + i;
        double2 v = to_d2(*ep);
        v.x += (J[q] - gauss) * INV4PI;
        *ep = from_d2<T>(v);
      }
    }
    __syncthreads();  // the queue is reused
  }
}

template <class T>
void launch_assemble(const int32_t* tb, const int32_t* m, const int32_t* sb, const int32_t* n,
                     const int64_t* off, int64_t nblk, const double* X, const double* Y,
                     const double* Z, const double* W, int kern, const double* k, T* pool,
                     const RegArgs* reg, hipStream_t s) {
  if (nblk <= 0) return;
  if (reg)
    hipLaunchKernelGGL(assemble_reg_kernel<T>, dim3((unsigned)nblk), dim3(WG), 0, s, tb, m, sb, n,
                       off, X, Y, Z, W, kern, k, pool, *reg);
  else
    hipLaunchKernelGGL(assemble_kernel<T>, dim3((unsigned)nblk), dim3(WG), 0, s, tb, m, sb, n, off,
                       X, Y, Z, W, kern, k, pool);
  HMX_LAUNCHED();
}

template void launch_assemble<double2>(const int32_t*, const int32_t*, const int32_t*,
                                       const int32_t*, const int64_t*, int64_t, const double*,
                                       const double*, const double*, const double*, int,
                                       const double*, double2*, const RegArgs*, hipStream_t);
template void launch_assemble<float2>(const int32_t*, const int32_t*, const int32_t*,
                                      const int32_t*, const int64_t*, int64_t, const double*,
                                      const double*, const double*, const double*, int,
                                      const double*, float2*, const RegArgs*, hipStream_t);

}  // namespace hmx

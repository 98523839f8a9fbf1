// k_matvec.hip -- the operator product y = K x.
//
// H-matrix product (row-leaf ownership; no floating-point atomics, fixed summation order):
//   1. gather     xp[p] = x[perm[p]]                           (cluster order)
//   2. far_vt     t_b = V_b^T xp[s_b] for every far block        (one workgroup per block)
//   3. leaf_apply for each leaf l:
//                 y_l = sum_{near b, row l} K_b xp[s_b] + sum_{far b, row node contains l}
//                       U_b[rows of l] t_b, written to y[perm[.]] (scatter fused)
// A far block stored dense is applied as U = K_b with t_b = xp[s_b].
//
// Dense product (operator built without a tolerance): every entry evaluated on the fly,
//   y_i = sum_l G(x_i, x_l) w_l x_l, as a 2-D grid of (64-row tile, 256-source chunk) partial
// sums, reduced over chunks in a fixed order.
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

// xp[i] = x[perm[i] - x_off] for the source points (original index >= x_off), 0 for the others
// (the target points of an operator between different point sets; x_off = 0 otherwise).
template <class T>
__global__ void gather_kernel(const T* __restrict__ x, const int32_t* __restrict__ perm,
                              T* __restrict__ xp, int64_t M, int64_t x_off) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < M) {
    const int64_t o = perm[i];
    xp[i] = o >= x_off ? x[o - x_off] : czero<T>();
  }
}

template <class T>
void launch_gather(const T* x, const int32_t* perm, T* xp, int64_t M, int64_t x_off,
                   hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel<T>, dim3((unsigned)((M + WG - 1) / WG)), dim3(WG), 0, s, x, perm,
                     xp, M, x_off);
  HMX_LAUNCHED();
}

__device__ __forceinline__ double2 wave_sum2(double2 v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}
__device__ __forceinline__ float2 wave_sum2(float2 v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}

// t_b[l] = sum_j V_b[j, l] xp[s_b + j]; wave w handles columns l = w, w + 4, ..., four (then two,
// then one) at a time, with the element loop unrolled, so that several column loads per lane are
// in flight (the kernel streams V from HBM)
template <class T>
__global__ void __launch_bounds__(WG) far_vt_kernel(const FarRec* __restrict__ rec,
                                                    const T* __restrict__ xp, T* __restrict__ t) {
  const FarRec f = rec[blockIdx.x];
  T* tb = t + f.toff;
  const T* xs = xp + f.sb;
  if (f.dense) {
    for (int j = threadIdx.x; j < f.n; j += WG) tb[j] = xs[j];
    return;
  }
  const int n = f.n, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t ldv = f.ldv;
  // column l of V: in the first segment below f.split, else in the second
  using gT = HMX_GLOBAL T;  // factor addresses read from the record: global space
  auto colv = [&](int l) -> const gT* {
    return l < f.split ? (const gT*)f.V + l * ldv : (const gT*)f.V1 + (l - f.split) * ldv;
  };
  int l = w;
  for (; l + 3 * NWAVE < f.r; l += 4 * NWAVE) {
    T a0 = czero<T>(), a1 = czero<T>(), a2 = czero<T>(), a3 = czero<T>();
    const gT* v0 = colv(l);
    const gT* v1 = colv(l + NWAVE);
    const gT* v2 = colv(l + 2 * NWAVE);
    const gT* v3 = colv(l + 3 * NWAVE);
#pragma unroll 2
    for (int j = lane; j < n; j += WAVE) {
      T xj = xs[j];
      cfma(a0, v0[j], xj);
      cfma(a1, v1[j], xj);
      cfma(a2, v2[j], xj);
      cfma(a3, v3[j], xj);
    }
    a0 = wave_sum2(a0);
    a1 = wave_sum2(a1);
    a2 = wave_sum2(a2);
    a3 = wave_sum2(a3);
    if (lane == 0) {
      tb[l] = a0;
      tb[l + NWAVE] = a1;
      tb[l + 2 * NWAVE] = a2;
      tb[l + 3 * NWAVE] = a3;
    }
  }
  for (; l + NWAVE < f.r; l += 2 * NWAVE) {
    T a0 = czero<T>(), a1 = czero<T>();
    const gT* v0 = colv(l);
    const gT* v1 = colv(l + NWAVE);
#pragma unroll 4
    for (int j = lane; j < n; j += WAVE) {
      T xj = xs[j];
      cfma(a0, v0[j], xj);
      cfma(a1, v1[j], xj);
    }
    a0 = wave_sum2(a0);
    a1 = wave_sum2(a1);
    if (lane == 0) {
      tb[l] = a0;
      tb[l + NWAVE] = a1;
    }
  }
  for (; l < f.r; l += NWAVE) {
    T a0 = czero<T>();
    const gT* v0 = colv(l);
#pragma unroll 4
    for (int j = lane; j < n; j += WAVE) cfma(a0, v0[j], xs[j]);
    a0 = wave_sum2(a0);
    if (lane == 0) tb[l] = a0;
  }
}

template <class T>
void launch_far_vt(const FarRec* rec, int64_t nf, const T* xp, T* t, hipStream_t s) {
  if (nf <= 0) return;
  hipLaunchKernelGGL(far_vt_kernel<T>, dim3((unsigned)nf), dim3(WG), 0, s, rec, xp, t);
  HMX_LAUNCHED();
}

constexpr int MAX_LEAF_CHUNKS = 4;  // rows per leaf <= 4 * 64

// The near field computed in the product (near_mode 1): the points and the kernel.
struct NearOtf {
  const double* X;
  const double* Y;
  const double* Z;
  const double* W;
  int kern;
  const double* kp;
};

// a[c] += sum_{l < nc} col_l[row[c]] tt[l], col_l = col + l ld (one segment of a far block's U).
// The factor address comes from the block record in memory, where the compiler cannot infer its
// space: as a global-space pointer its loads count only against the vector-memory counter, so
// the scalar loads of tt do not wait for them.
template <class T, int NCH>
__device__ __forceinline__ void far_cols(T (&a)[NCH], const int (&row)[NCH], const T* colp,
                                         int64_t ld, const T* __restrict__ tt, int nc) {
  constexpr int UNR = 8 / NCH;  // columns per unrolled round (8 loads in flight per lane)
  using gT = HMX_GLOBAL T;
  const gT* col = (const gT*)colp;
#pragma unroll UNR
  for (int l = 0; l < nc; ++l, col += ld) {
    const T tl = tt[l];
#pragma unroll
    for (int c = 0; c < NCH; ++c) cfma(a[c], col[row[c]], tl);
  }
}

// The stored blocks of one leaf of m <= NCH * 64 rows, for wave w: near blocks it = w, w + 4, ...
// below nn, then far blocks, accumulated into acc[c] (row lane + 64 c).  The loads carry no
// condition: lanes past the leaf's rows read its last row and their sums are discarded, so
// that 8 / NCH columns of NCH loads each can be in flight per wave.
template <class T, int NCH, int MAXCH>
__device__ __forceinline__ void leaf_blocks(
    T (&acc)[MAXCH], int lane, int w, int m, int tb, int64_t n0, int64_t nn,
    int64_t f0, int64_t nfar, const int32_t* __restrict__ near_sb,
    const int32_t* __restrict__ near_n, const int64_t* __restrict__ near_off,
    const T* __restrict__ near_pool, const int32_t* __restrict__ far_list,
    const FarRec* __restrict__ far, const T* __restrict__ tbuf, const T* __restrict__ xp) {
  constexpr int UNR = 8 / NCH;  // near-block columns per unrolled round
  T a[NCH];
  int row[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    a[c] = acc[c];
    row[c] = min(lane + c * WAVE, m - 1);
  }
  for (int64_t it = w; it < nn + nfar; it += NWAVE) {
    if (it < nn) {
      const int64_t blk = n0 + it;
      const int sb = near_sb[blk], n = near_n[blk];
      const T* K = near_pool + near_off[blk];
      const T* xs = xp + sb;
#pragma unroll UNR
      for (int j = 0; j < n; ++j) {
        const T xj = xs[j];
        const T* col = K + (int64_t)j * m;
#pragma unroll
        for (int c = 0; c < NCH; ++c) cfma(a[c], col[row[c]], xj);
      }
    } else {
      const FarRec f = far[far_list[f0 + (it - nn)]];
      const int o = tb - f.tb;
      const T* tt = tbuf + f.toff;
      // columns below f.split in the first segment of U, the rest in the second
      const int r0 = min(f.r, f.split);
      far_cols<T, NCH>(a, row, (const T*)f.U + o, f.ldu, tt, r0);
      far_cols<T, NCH>(a, row, (const T*)f.U1 + o, f.ldu, tt + r0, f.r - r0);
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = lane + c * WAVE < m ? a[c] : czero<T>();
}

// OTF = false: near blocks read from near_pool.  OTF = true: near blocks evaluated here.  For each
// near block of the leaf in turn, the workgroup stages the block's source points and x entries
// in LDS (one per thread), then wave w evaluates the sources j = w, w + 4, ... against all of
// the leaf's rows (targets kept in registers), accumulating K_ij x_j; the far blocks follow as
// in the stored case.  Each row's terms are summed per wave in a fixed order, then over the
// waves, so the product is deterministic.
// MAXCH: 64-row chunks of the largest leaf (the kernel's registers and LDS are sized for it).
template <class T, bool OTF, int MAXCH>
__global__ void __launch_bounds__(WG) leaf_apply_kernel(
    const int32_t* __restrict__ leaves, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const int64_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_sb, const int32_t* __restrict__ near_n,
    const int64_t* __restrict__ near_off, const T* __restrict__ near_pool,
    const int64_t* __restrict__ far_ptr, const int32_t* __restrict__ far_list,
    const FarRec* __restrict__ far, const T* __restrict__ tbuf,
    const T* __restrict__ xp, const int32_t* __restrict__ perm, int64_t y_rows,
    T* __restrict__ y, NearOtf otf) {
  __shared__ T part[NWAVE][MAXCH * WAVE];
  const int leaf = blockIdx.x;
  const int node = leaves[leaf];
  const int tb = nbegin[node], m = nend[node] - tb;
  const int64_t n0 = near_ptr[leaf], nn_all = near_ptr[leaf + 1] - n0;
  const int64_t f0 = far_ptr[leaf], nfar = far_ptr[leaf + 1] - f0;
  // the wave index is uniform across the wave: marked so, the block descriptors and the
  // x and t entries, whose addresses depend only on it, are read through scalar loads
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int nch = (m + WAVE - 1) / WAVE;
  T acc[MAXCH];
#pragma unroll
  for (int c = 0; c < MAXCH; ++c) acc[c] = czero<T>();
  int64_t nn = nn_all;  // near blocks left to the per-wave loops below
  if constexpr (OTF) {
    constexpr int TILE = MAXCH * WAVE;  // a near block's sources (a leaf)
    __shared__ double spt[4][TILE];              // source x, y, z, w
    __shared__ T sxp[TILE];                      // source entries of x
    const double k = otf.kp[tb];
    double tx[MAXCH], ty[MAXCH], tz[MAXCH];
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
      const int i = min(lane + c * WAVE, m - 1);
      tx[c] = otf.X[tb + i];
      ty[c] = otf.Y[tb + i];
      tz[c] = otf.Z[tb + i];
    }
    for (int64_t b = 0; b < nn_all; ++b) {
      const int64_t blk = n0 + b;
      const int sb = near_sb[blk], n = near_n[blk];
      for (int j = threadIdx.x; j < n; j += WG) {
        spt[0][j] = otf.X[sb + j];
        spt[1][j] = otf.Y[sb + j];
        spt[2][j] = otf.Z[sb + j];
        spt[3][j] = otf.W[sb + j];
        sxp[j] = xp[sb + j];
      }
      __syncthreads();
      for (int j = w; j < n; j += NWAVE) {
        const double sx = spt[0][j], sy = spt[1][j], sz = spt[2][j], sw = spt[3][j];
        const T xj = sxp[j];
#pragma unroll
        for (int c = 0; c < MAXCH; ++c) {
          if (c < nch) {
            const T g = eval_entry<T>(otf.kern, k, tx[c], ty[c], tz[c], sx, sy, sz, sw);
            cfma(acc[c], g, xj);
          }
        }
      }
      __syncthreads();  // the tile is read by every wave before the next block replaces it
    }
    nn = 0;
  }
  if (MAXCH == 1 || nch == 1)
    leaf_blocks<T, 1, MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb, near_n, near_off,
                             near_pool, far_list, far, tbuf, xp);
  else if (MAXCH == 2 || nch == 2)
    leaf_blocks<T, (MAXCH < 2 ? MAXCH : 2), MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb,
                                                   near_n, near_off, near_pool, far_list, far,
                                                   tbuf, xp);
  else if (MAXCH == 3 || nch == 3)
    leaf_blocks<T, (MAXCH < 3 ? MAXCH : 3), MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb,
                                                   near_n, near_off, near_pool, far_list, far,
                                                   tbuf, xp);
  else
    leaf_blocks<T, MAXCH, MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb, near_n, near_off,
                                 near_pool, far_list, far, tbuf, xp);
#pragma unroll
  for (int c = 0; c < MAXCH; ++c) part[w][lane + c * WAVE] = acc[c];
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += WG) {
    T s = part[0][i];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) {
      s.x += part[q][i].x;
      s.y += part[q][i].y;
    }
    const int64_t o = perm[tb + i];
    if (o < y_rows) y[o] = s;  // rows of the product only (not the sources of a
                               // different-point-set operator)
  }
}

template <class T, bool OTF, int MAXCH>
void leaf_apply_launch(int n_leaves, const int32_t* leaves, const int32_t* nbegin,
                       const int32_t* nend, const int64_t* near_ptr, const int32_t* near_sb,
                       const int32_t* near_n, const int64_t* near_off, const T* near_pool,
                       const int64_t* far_ptr, const int32_t* far_list, const FarRec* far,
                       const T* tbuf, const T* xp, const int32_t* perm, int64_t y_rows, T* y,
                       hipStream_t s, const NearOtf& o) {
  hipLaunchKernelGGL((leaf_apply_kernel<T, OTF, MAXCH>), dim3(n_leaves), dim3(WG), 0, s, leaves,
                     nbegin, nend, near_ptr, near_sb, near_n, near_off, near_pool, far_ptr,
                     far_list, far, tbuf, xp, perm, y_rows, y, o);
  HMX_LAUNCHED();
}

template <class T>
void launch_leaf_apply(int n_leaves, const int32_t* leaves, const int32_t* nbegin,
                       const int32_t* nend, const int64_t* near_ptr, const int32_t* near_sb,
                       const int32_t* near_n, const int64_t* near_off, const T* near_pool,
                       const int64_t* far_ptr, const int32_t* far_list, const FarRec* far,
                       const T* tbuf, const T* xp, const int32_t* perm, int64_t y_rows, T* y,
                       int max_leaf_rows, hipStream_t s, const NearOtfArgs* otf) {
  if (n_leaves <= 0) return;
  HMX_REQUIRE(max_leaf_rows >= 1 && max_leaf_rows <= MAX_LEAF_CHUNKS * WAVE, HMX_EINTERNAL,
              "leaf rows outside [1, 256]");
  NearOtf o{};
  if (otf) o = NearOtf{otf->X, otf->Y, otf->Z, otf->W, otf->kern, otf->kp};
  int ch = (max_leaf_rows + WAVE - 1) / WAVE;
  // FP64 with the near field on the fly: the two-chunk instance runs 64-row leaves about 5 %
  // faster than the one-chunk one (measured; same arithmetic, same order), so it takes them too
  if (otf && sizeof(T) == 16 && ch == 1) ch = 2;
#define HMX_LEAF_LAUNCH(OTF, CH)                                                                 \
  leaf_apply_launch<T, OTF, CH>(n_leaves, leaves, nbegin, nend, near_ptr, near_sb, near_n,       \
                                near_off, near_pool, far_ptr, far_list, far, tbuf, xp, perm,     \
                                y_rows, y, s, o)
  if (otf) {
    if (ch == 1) HMX_LEAF_LAUNCH(true, 1);
    else if (ch == 2) HMX_LEAF_LAUNCH(true, 2);
    else HMX_LEAF_LAUNCH(true, 4);
  } else {
    if (ch == 1) HMX_LEAF_LAUNCH(false, 1);
    else if (ch == 2) HMX_LEAF_LAUNCH(false, 2);
    else HMX_LEAF_LAUNCH(false, 4);
  }
#undef HMX_LEAF_LAUNCH
}

// ---------------------------------------------------------- several vectors at once (NR = 2, 4)
// The same product for NR vectors: vector r of xp and t at offset r ldx and r ldt, output r to
// y.p[r].  Every entry of V, U and the near blocks is loaded once and applied to the NR vectors,
// so the operator's bytes are read once for all of them; the summation order per vector is that
// of the one-vector kernels' general paths (one column, or one near-block column, at a time).
template <class T>
struct MultiOut {
  T* p[4];
};

template <class T, int NR>
__global__ void __launch_bounds__(WG) far_vt_multi_kernel(const FarRec* __restrict__ rec,
                                                          const T* __restrict__ xp, int64_t ldx,
                                                          T* __restrict__ t, int64_t ldt) {
  const FarRec f = rec[blockIdx.x];
  T* tb = t + f.toff;
  const T* xs = xp + f.sb;
  if (f.dense) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      for (int j = threadIdx.x; j < f.n; j += WG) tb[r * ldt + j] = xs[r * ldx + j];
    return;
  }
  const int n = f.n, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t ldv = f.ldv;
  using gT = HMX_GLOBAL T;  // factor addresses read from the record: global space
  auto colv = [&](int l) -> const gT* {
    return l < f.split ? (const gT*)f.V + l * ldv : (const gT*)f.V1 + (l - f.split) * ldv;
  };
  int l = w;
  for (; l + 3 * NWAVE < f.r; l += 4 * NWAVE) {
    T a[4][NR];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) a[c][r] = czero<T>();
    const gT* v[4] = {colv(l), colv(l + NWAVE), colv(l + 2 * NWAVE), colv(l + 3 * NWAVE)};
    for (int j = lane; j < n; j += WAVE) {
      T p[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) p[c] = v[c][j];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const T xj = xs[r * ldx + j];
#pragma unroll
        for (int c = 0; c < 4; ++c) cfma(a[c][r], p[c], xj);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        a[c][r] = wave_sum2(a[c][r]);
        if (lane == 0) tb[r * ldt + l + c * NWAVE] = a[c][r];
      }
  }
  for (; l + NWAVE < f.r; l += 2 * NWAVE) {
    T a0[NR], a1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) a0[r] = a1[r] = czero<T>();
    const gT* v0 = colv(l);
    const gT* v1 = colv(l + NWAVE);
#pragma unroll 2
    for (int j = lane; j < n; j += WAVE) {
      const T p0 = v0[j], p1 = v1[j];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const T xj = xs[r * ldx + j];
        cfma(a0[r], p0, xj);
        cfma(a1[r], p1, xj);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      a0[r] = wave_sum2(a0[r]);
      a1[r] = wave_sum2(a1[r]);
      if (lane == 0) {
        tb[r * ldt + l] = a0[r];
        tb[r * ldt + l + NWAVE] = a1[r];
      }
    }
  }
  for (; l < f.r; l += NWAVE) {
    T a0[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) a0[r] = czero<T>();
    const gT* v0 = colv(l);
#pragma unroll 2
    for (int j = lane; j < n; j += WAVE) {
      const T p0 = v0[j];
#pragma unroll
      for (int r = 0; r < NR; ++r) cfma(a0[r], p0, xs[r * ldx + j]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      a0[r] = wave_sum2(a0[r]);
      if (lane == 0) tb[r * ldt + l] = a0[r];
    }
  }
}

// a[c][r] += sum_{l < nc} col_l[row[c]] tt[r ldt + l], col_l = col + l ld (one segment of U).
template <class T, int NR, int NCH>
__device__ __forceinline__ void far_cols_multi(T (&a)[NCH][NR], const int (&row)[NCH],
                                               const T* colp, int64_t ld,
                                               const T* __restrict__ tt, int64_t ldt, int nc) {
  constexpr int UNR = NCH < 4 ? 4 / NCH : 1;  // columns per unrolled round
  using gT = HMX_GLOBAL T;
  const gT* col = (const gT*)colp;
#pragma unroll UNR
  for (int l = 0; l < nc; ++l, col += ld) {
    T tl[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tl[r] = tt[r * ldt + l];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const T uil = col[row[c]];
#pragma unroll
      for (int r = 0; r < NR; ++r) cfma(a[c][r], uil, tl[r]);
    }
  }
}

// The blocks of one leaf for NR vectors, as leaf_blocks does for one: the same order of sums per
// vector, condition-free loads (lanes past the leaf's rows read its last row and drop the sums).
template <class T, int NR, int NCH, int MAXCH>
__device__ __forceinline__ void leaf_blocks_multi(
    T (&acc)[MAXCH][NR], int lane, int w, int m, int tb, int64_t n0, int64_t nn, int64_t f0,
    int64_t nfar, const int32_t* __restrict__ near_sb, const int32_t* __restrict__ near_n,
    const int64_t* __restrict__ near_off, const T* __restrict__ near_pool,
    const int32_t* __restrict__ far_list, const FarRec* __restrict__ far,
    const T* __restrict__ tbuf, int64_t ldt, const T* __restrict__ xp, int64_t ldx) {
  constexpr int UNR = NCH < 4 ? 4 / NCH : 1;  // near-block columns per unrolled round
  T a[NCH][NR];
  int row[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    row[c] = min(lane + c * WAVE, m - 1);
#pragma unroll
    for (int r = 0; r < NR; ++r) a[c][r] = czero<T>();
  }
  for (int64_t it = w; it < nn + nfar; it += NWAVE) {
    if (it < nn) {
      const int64_t blk = n0 + it;
      const int sb = near_sb[blk], n = near_n[blk];
      const T* K = near_pool + near_off[blk];
      const T* xs = xp + sb;
#pragma unroll UNR
      for (int j = 0; j < n; ++j) {
        T xj[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) xj[r] = xs[r * ldx + j];
        const T* col = K + (int64_t)j * m;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const T kij = col[row[c]];
#pragma unroll
          for (int r = 0; r < NR; ++r) cfma(a[c][r], kij, xj[r]);
        }
      }
    } else {
      const FarRec f = far[far_list[f0 + (it - nn)]];
      const int o = tb - f.tb;
      const T* tt = tbuf + f.toff;
      // columns below f.split in the first segment of U, the rest in the second
      const int r0 = min(f.r, f.split);
      far_cols_multi<T, NR, NCH>(a, row, (const T*)f.U + o, f.ldu, tt, ldt, r0);
      far_cols_multi<T, NR, NCH>(a, row, (const T*)f.U1 + o, f.ldu, tt + r0, ldt, f.r - r0);
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const bool on = lane + c * WAVE < m;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[c][r] = on ? a[c][r] : czero<T>();
  }
}

// MAXCH: 64-row chunks of the largest leaf, as in leaf_apply_kernel.
template <class T, int NR, int MAXCH>
__global__ void __launch_bounds__(WG) leaf_apply_multi_kernel(
    const int32_t* __restrict__ leaves, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const int64_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_sb, const int32_t* __restrict__ near_n,
    const int64_t* __restrict__ near_off, const T* __restrict__ near_pool,
    const int64_t* __restrict__ far_ptr, const int32_t* __restrict__ far_list,
    const FarRec* __restrict__ far, const T* __restrict__ tbuf, int64_t ldt,
    const T* __restrict__ xp, int64_t ldx, const int32_t* __restrict__ perm, int64_t y_rows,
    MultiOut<T> y) {
  __shared__ T part[NWAVE][MAXCH * WAVE];
  const int leaf = blockIdx.x;
  const int node = leaves[leaf];
  const int tb = nbegin[node], m = nend[node] - tb;
  const int64_t n0 = near_ptr[leaf], nn = near_ptr[leaf + 1] - n0;
  const int64_t f0 = far_ptr[leaf], nfar = far_ptr[leaf + 1] - f0;
  // the wave index is uniform across the wave: marked so, the block descriptors and the
  // x and t entries, whose addresses depend only on it, are read through scalar loads
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int nch = (m + WAVE - 1) / WAVE;
  T acc[MAXCH][NR];
#pragma unroll
  for (int c = 0; c < MAXCH; ++c)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[c][r] = czero<T>();
  if (MAXCH == 1 || nch == 1)
    leaf_blocks_multi<T, NR, 1, MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb, near_n,
                                       near_off, near_pool, far_list, far, tbuf, ldt, xp, ldx);
  else if (MAXCH == 2 || nch == 2)
    leaf_blocks_multi<T, NR, (MAXCH < 2 ? MAXCH : 2), MAXCH>(acc, lane, w, m, tb, n0, nn, f0,
                                                             nfar, near_sb, near_n, near_off,
                                                             near_pool, far_list, far, tbuf, ldt,
                                                             xp, ldx);
  else if (MAXCH == 3 || nch == 3)
    leaf_blocks_multi<T, NR, (MAXCH < 3 ? MAXCH : 3), MAXCH>(acc, lane, w, m, tb, n0, nn, f0,
                                                             nfar, near_sb, near_n, near_off,
                                                             near_pool, far_list, far, tbuf, ldt,
                                                             xp, ldx);
  else
    leaf_blocks_multi<T, NR, MAXCH, MAXCH>(acc, lane, w, m, tb, n0, nn, f0, nfar, near_sb, near_n,
                                           near_off, near_pool, far_list, far, tbuf, ldt, xp,
                                           ldx);
  // one vector at a time through the same LDS buffer
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) part[w][lane + c * WAVE] = acc[c][r];
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += WG) {
      T s = part[0][i];
#pragma unroll
      for (int q = 1; q < NWAVE; ++q) {
        s.x += part[q][i].x;
        s.y += part[q][i].y;
      }
      const int64_t o = perm[tb + i];
      if (o < y_rows) y.p[r][o] = s;
    }
    __syncthreads();
  }
}

// y_r = K x_r for r < nr (nr = 2 or 4): x_r, y_r device vectors of the product's shape; xpm holds
// nr M and tm nr t_len entries of scratch.
template <class T>
void launch_matvec_multi(const hmx_op* op, int nr, const T* const* x, T* const* y, T* xpm, T* tm,
                         hipStream_t s) {
  const int64_t M = op->M, ldt = std::max<int64_t>(op->t_len, 1);
  HMX_REQUIRE(op->max_leaf_rows >= 1 && op->max_leaf_rows <= MAX_LEAF_CHUNKS * WAVE,
              HMX_EINTERNAL, "leaf rows outside [1, 256]");
  const int ch = (op->max_leaf_rows + WAVE - 1) / WAVE;
  MultiOut<T> out{};
  for (int r = 0; r < nr; ++r) {
    launch_gather<T>(x[r], op->perm.p, xpm + r * M, M, op->x_off, s);
    out.p[r] = y[r];
  }
  auto go = [&](auto nrc) {
    constexpr int NR = decltype(nrc)::value;
    if (op->n_far > 0) {
      hipLaunchKernelGGL((far_vt_multi_kernel<T, NR>), dim3((unsigned)op->n_far), dim3(WG), 0, s,
                         op->far.p, xpm, M, tm, ldt);
      HMX_LAUNCHED();
    }
    auto leaves = [&](auto chc) {
      constexpr int CH = decltype(chc)::value;
      hipLaunchKernelGGL((leaf_apply_multi_kernel<T, NR, CH>), dim3(op->n_leaves), dim3(WG), 0,
                         s, op->leaves.p, op->nbegin.p, op->nend.p, op->near_ptr.p,
                         op->near_sb.p, op->near_n.p, op->near_off.p, (const T*)op->near_pool.p,
                         op->far_ptr.p, op->far_list.p, op->far.p, tm, ldt, xpm, M, op->perm.p,
                         op->rows, out);
      HMX_LAUNCHED();
    };
    if (op->n_leaves <= 0) return;
    if (ch == 1)
      leaves(std::integral_constant<int, 1>{});
    else if (ch == 2)
      leaves(std::integral_constant<int, 2>{});
    else
      leaves(std::integral_constant<int, 4>{});
  };
  if (nr == 2)
    go(std::integral_constant<int, 2>{});
  else if (nr == 4)
    go(std::integral_constant<int, 4>{});
  else
    throw Error(HMX_EINTERNAL, "launch_matvec_multi: nr must be 2 or 4");
}

// ------------------------------------------------------------------------- dense on the fly
constexpr int DOTF_CHUNK = 256;  // sources per workgroup (64 per wavefront)

int64_t dense_otf_partial_len(int64_t rows, int64_t cols) {
  int64_t nch = (cols + DOTF_CHUNK - 1) / DOTF_CHUNK;
  return nch * rows;
}

// Rows are the points [0, rows), columns the points [so, so + cols) with x indexed from 0
// (square operators: rows = cols = M, so = 0).
template <class T>
__global__ void __launch_bounds__(WG) dense_otf_kernel(const double* __restrict__ X,
                                                       const double* __restrict__ Y,
                                                       const double* __restrict__ Z,
                                                       const double* __restrict__ W, int64_t rows,
                                                       int64_t so, int64_t cols, int kern, double k,
                                                       const T* __restrict__ x,
                                                       T* __restrict__ partial) {
  __shared__ T part[NWAVE][WAVE];
  // the wavefront index is uniform, so the source loop and its loads (one source for all 64
  // lanes) run on the scalar unit
  const int lane = threadIdx.x & (WAVE - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t i = (int64_t)blockIdx.x * WAVE + lane;
  const int64_t j0 = (int64_t)blockIdx.y * DOTF_CHUNK + w * WAVE;
  const int64_t j1 = min(j0 + WAVE, cols);
  T acc = czero<T>();
  if (i < rows) {
    const double tx = X[i], ty = Y[i], tz = Z[i];
    for (int64_t j = j0; j < j1; ++j) {
      T g = eval_entry<T>(kern, k, tx, ty, tz, X[so + j], Y[so + j], Z[so + j], W[so + j]);
      cfma(acc, g, x[j]);
    }
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < rows) {
    T s = part[0][lane];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) {
      s.x += part[q][lane].x;
      s.y += part[q][lane].y;
    }
    partial[(int64_t)blockIdx.y * rows + i] = s;
  }
}

template <class T>
__global__ void dense_reduce_kernel(const T* __restrict__ partial, int64_t nch, int64_t M,
                                    T* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= M) return;
  T s = partial[i];
  for (int64_t c = 1; c < nch; ++c) {
    T v = partial[c * M + i];
    s.x += v.x;
    s.y += v.y;
  }
  y[i] = s;
}

template <class T>
void launch_dense_otf(const double* X, const double* Y, const double* Z, const double* W,
                      int64_t rows, int64_t so, int64_t cols, int kern, double k, const T* x,
                      T* partial, T* y, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  int64_t nrt = (rows + WAVE - 1) / WAVE, nch = (cols + DOTF_CHUNK - 1) / DOTF_CHUNK;
  hipLaunchKernelGGL(dense_otf_kernel<T>, dim3((unsigned)nrt, (unsigned)nch), dim3(WG), 0, s, X, Y,
                     Z, W, rows, so, cols, kern, k, x, partial);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(dense_reduce_kernel<T>, dim3((unsigned)((rows + WG - 1) / WG)), dim3(WG), 0, s,
                     partial, nch, rows, y);
  HMX_LAUNCHED();
}

#define HMX_INST(T)                                                                              \
  template void launch_gather<T>(const T*, const int32_t*, T*, int64_t, int64_t, hipStream_t);   \
  template void launch_far_vt<T>(const FarRec*, int64_t, const T*, T*, hipStream_t);             \
  template void launch_leaf_apply<T>(int, const int32_t*, const int32_t*, const int32_t*,        \
                                     const int64_t*, const int32_t*, const int32_t*,             \
                                     const int64_t*, const T*, const int64_t*, const int32_t*,   \
                                     const FarRec*, const T*, const T*, const int32_t*, int64_t, \
                                     T*, int, hipStream_t, const NearOtfArgs*);                  \
  template void launch_dense_otf<T>(const double*, const double*, const double*, const double*,  \
                                    int64_t, int64_t, int64_t, int, double, const T*, T*, T*,    \
                                    hipStream_t);                                                \
  template void launch_matvec_multi<T>(const hmx_op*, int, const T* const*, T* const*, T*, T*,   \
                                       hipStream_t);
HMX_INST(double2)
HMX_INST(float2)
#undef HMX_INST

}  // namespace hmx

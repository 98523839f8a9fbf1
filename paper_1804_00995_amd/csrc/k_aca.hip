// k_aca.hip -- partially pivoted adaptive cross approximation of the far blocks.
//
// The paper compresses the kernel matrix "to the desired tolerance" without stating the method;
// libhmx uses Bebendorf-style partial pivoting.  For a far block A (m x n, A_ij =
// G(x_{t+i}, x_{s+j}) w_{s+j}), step k with pivot row i_k:
//   (1) residual row R_j = A(i_k, j) - sum_{l<k} u_l[i_k] v_l[j]
//   (2) pivot column j_k = argmax over unused columns of |R_j|^2 (lowest index on ties); a row
//       whose residual maximum is <= 1e-300 is marked used, the lowest unused row is taken and
//       no term is added
//   (3) v_k = R / R_{j_k}
//   (4) u_k[i] = A(i, j_k) - sum_{l<k} v_l[j_k] u_l[i]
//   (5) |S_k|_F^2 = |S_{k-1}|_F^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k) + |u_k|^2 |v_k|^2
//   (6) stop, keeping term k, when |u_k| |v_k| <= tol |S_k|_F
//   (7) next pivot row = argmax over unused rows of |u_k[i]|^2 (lowest index on ties).
// A ~ sum_k u_k v_k^T with U (m x cap) and V (n x cap) stored column-major.  Pivot magnitudes,
// norms and the cross terms are accumulated in FP64 in both precisions.
//
// Schedule: a persistent grid; each 256-thread workgroup takes the next block from an atomic
// counter (blocks pre-ordered by decreasing size) and runs its whole sequential step chain.
// A block that needs a term beyond its slot capacity saves (rank, pivot row, norm) and stops
// with status OVERFLOW; the host gives it a larger slot and the kernel continues from the saved
// state, so the sequence of pivots, and therefore the factors, are the same as in one run.
// A block that needs a term beyond its rank cap is marked DENSE (stored exactly).
#include <limits.h>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

template <class T>
__device__ void aca_block(const FarDesc& d, int b, const double* __restrict__ X,
                          const double* __restrict__ Y, const double* __restrict__ Z,
                          const double* __restrict__ W, int kern, double k, double tol,
                          uint8_t* flags, int32_t* rank, int32_t* ipiv, int32_t* status,
                          double* norm2, int fresh, T* coef, double* sv, int* si, double* ssum) {
  const int tid = threadIdx.x;
  const int m = d.m, n = d.n, tb = d.tb, sb = d.sb;
  T* U = (T*)d.U;
  T* V = (T*)d.V;
  uint8_t* rused = flags + d.foff;
  uint8_t* cused = rused + m;
  int kk, ip;
  double nrm2;
  if (fresh) {
    for (int i = tid; i < m + n; i += WG) rused[i] = 0;
    kk = 0;
    ip = 0;
    nrm2 = 0.0;
  } else {
    kk = rank[b];
    ip = ipiv[b];
    nrm2 = norm2[b];
  }
  __syncthreads();
  int st = d.rcap <= 0 ? ACA_DENSE : ACA_RUNNING;
  while (st == ACA_RUNNING) {
    // (1) residual row ip, stored as column kk of V when the slot has room
    for (int l = tid; l < kk; l += WG) coef[l] = U[(int64_t)l * m + ip];
    __syncthreads();
    const double px = X[tb + ip], py = Y[tb + ip], pz = Z[tb + ip];
    const bool store = kk < d.cap;
    T* R = V + (int64_t)kk * n;
    double best = -1.0;
    int bj = INT_MAX;
    for (int j = tid; j < n; j += WG) {
      T a = eval_entry<T>(kern, k, px, py, pz, X[sb + j], Y[sb + j], Z[sb + j], W[sb + j]);
      for (int l = 0; l < kk; ++l) cfms(a, coef[l], V[(int64_t)l * n + j]);
      if (store) R[j] = a;
      if (!cused[j]) amax_merge(best, bj, abs2(a), j);
    }
    block_amax(best, bj, sv, si);
    if (bj == INT_MAX || best <= 1e-300) {
      // (2') zero residual row: mark it, move to the lowest unused row
      if (tid == 0) rused[ip] = 1;
      __syncthreads();
      int nx = INT_MAX;
      for (int i = tid; i < m; i += WG)
        if (!rused[i]) {
          nx = i;
          break;
        }
      nx = block_min(nx, si);
      if (nx == INT_MAX) {
        st = ACA_CONVERGED;
        break;
      }
      ip = nx;
      continue;
    }
    if (!store) {
      st = d.cap >= d.rcap ? ACA_DENSE : ACA_OVERFLOW;
      break;
    }
    // (3) v_k = R / R[bj]
    const double2 pd = to_d2(R[bj]);
    const double den = pd.x * pd.x + pd.y * pd.y;
    const T inv = from_d2<T>(make_double2(pd.x / den, -pd.y / den));
    __syncthreads();  // every thread has read the pivot before it is scaled in place
    if (tid == 0) {
      rused[ip] = 1;
      cused[bj] = 1;
    }
    double nv2 = 0.0;
    for (int j = tid; j < n; j += WG) {
      T v = cmul(R[j], inv);
      R[j] = v;
      nv2 += abs2(v);
    }
    __syncthreads();
    // (4) residual column bj, stored as column kk of U
    for (int l = tid; l < kk; l += WG) coef[l] = V[(int64_t)l * n + bj];
    __syncthreads();
    const double qx = X[sb + bj], qy = Y[sb + bj], qz = Z[sb + bj], qw = W[sb + bj];
    T* Uk = U + (int64_t)kk * m;
    double ub = -1.0, nu2 = 0.0;
    int ui = INT_MAX;
    for (int i = tid; i < m; i += WG) {
      T a = eval_entry<T>(kern, k, X[tb + i], Y[tb + i], Z[tb + i], qx, qy, qz, qw);
      for (int l = 0; l < kk; ++l) cfms(a, coef[l], U[(int64_t)l * m + i]);
      Uk[i] = a;
      double a2 = abs2(a);
      nu2 += a2;
      if (!rused[i]) amax_merge(ub, ui, a2, i);
    }
    __syncthreads();
    // (5) cross terms sum_{l<kk} (u_l^H u_k)(v_l^H v_k), four l at a time
    double cross = 0.0;
    for (int l0 = 0; l0 < kk; l0 += 4) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      for (int i = tid; i < m; i += WG) {
        double2 uk = to_d2(Uk[i]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (l0 + q < kk) {
            double2 ul = to_d2(U[(int64_t)(l0 + q) * m + i]);
            acc[2 * q] += ul.x * uk.x + ul.y * uk.y;
            acc[2 * q + 1] += ul.x * uk.y - ul.y * uk.x;
          }
        }
      }
      for (int j = tid; j < n; j += WG) {
        double2 vk = to_d2(R[j]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (l0 + q < kk) {
            double2 vl = to_d2(V[(int64_t)(l0 + q) * n + j]);
            acc[8 + 2 * q] += vl.x * vk.x + vl.y * vk.y;
            acc[8 + 2 * q + 1] += vl.x * vk.y - vl.y * vk.x;
          }
        }
      }
      block_sum<16>(acc, ssum);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (l0 + q < kk) cross += acc[2 * q] * acc[8 + 2 * q] - acc[2 * q + 1] * acc[8 + 2 * q + 1];
    }
    double nn2[2] = {nu2, nv2};
    block_sum<2>(nn2, ssum);
    nrm2 = nrm2 + 2.0 * cross + nn2[0] * nn2[1];
    kk += 1;
    block_amax(ub, ui, sv, si);
    // (6) stopping rule, (7) next pivot row
    if (sqrt(nn2[0]) * sqrt(nn2[1]) <= tol * sqrt(nrm2)) {
      st = ACA_CONVERGED;
      break;
    }
    if (ui == INT_MAX) {
      st = ACA_CONVERGED;
      break;
    }
    ip = ui;
  }
  if (tid == 0) {
    rank[b] = kk;
    ipiv[b] = ip;
    norm2[b] = nrm2;
    status[b] = st;
  }
  __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(WG) aca_kernel(const FarDesc* __restrict__ desc,
                                                 const int32_t* __restrict__ order, int nb,
                                                 int* counter, const double* __restrict__ X,
                                                 const double* __restrict__ Y,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ W, int kern, double k,
                                                 double tol, uint8_t* flags, int32_t* rank,
                                                 int32_t* ipiv, int32_t* status, double* norm2,
                                                 int fresh) {
  __shared__ T coef[ACA_COEF_MAX];
  __shared__ double sv[NWAVE];
  __shared__ int si[NWAVE];
  __shared__ double ssum[16 * NWAVE];
  __shared__ int s_q;
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(counter, 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= nb) break;
    const int b = order[q];
    const FarDesc d = desc[b];
    aca_block<T>(d, b, X, Y, Z, W, kern, k, tol, flags, rank, ipiv, status, norm2, fresh,
                 coef, sv, si, ssum);
  }
}

template <class T>
void launch_aca(const FarDesc* d, const int32_t* order, int nb, int* counter, const double* X,
                const double* Y, const double* Z, const double* W, int kern, double k, double tol,
                uint8_t* flags, int32_t* rank, int32_t* ipiv, int32_t* status, double* norm2,
                int fresh, hipStream_t s) {
  if (nb <= 0) return;
  int dev = 0, ncu = 0;
  HMX_HIP(hipGetDevice(&dev));
  HMX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int per_cu = 0;
  HMX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, aca_kernel<T>, WG, 0));
  if (per_cu < 1) per_cu = 1;
  int grid = ncu * per_cu;
  if (grid > nb) grid = nb;
  hipLaunchKernelGGL(aca_kernel<T>, dim3(grid), dim3(WG), 0, s, d, order, nb, counter, X, Y, Z, W,
                     kern, k, tol, flags, rank, ipiv, status, norm2, fresh);
  HMX_LAUNCHED();
}

// Copy the first rank[b] columns of U and V of listed blocks from their old slot to a new one
// (both column-major with the same leading dimension, so each factor is one contiguous run).
template <class T>
__global__ void __launch_bounds__(WG) copy_factors_kernel(const FarDesc* __restrict__ from,
                                                          const FarDesc* __restrict__ to,
                                                          const int32_t* __restrict__ rank,
                                                          const int32_t* __restrict__ list) {
  const int b = list[blockIdx.x];
  const FarDesc a = from[b], c = to[b];
  const int64_t r = rank[b];
  const int64_t nu = r * a.m, nv = r * a.n;
  const T* su = (const T*)a.U;
  const T* sv = (const T*)a.V;
  T* du = (T*)c.U;
  T* dv = (T*)c.V;
  for (int64_t e = threadIdx.x; e < nu; e += WG) du[e] = su[e];
  for (int64_t e = threadIdx.x; e < nv; e += WG) dv[e] = sv[e];
}

template <class T>
void launch_copy_factors(const FarDesc* from, const FarDesc* to, const int32_t* rank,
                         const int32_t* list, int nlist, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(copy_factors_kernel<T>, dim3(nlist), dim3(WG), 0, s, from, to, rank, list);
  HMX_LAUNCHED();
}

// Final compaction: low-rank blocks' U (m x r) and V (n x r) into their final offsets.
template <class T>
__global__ void __launch_bounds__(WG) compact_kernel(const FarDesc* __restrict__ d,
                                                     const FarRec* __restrict__ rec,
                                                     const int32_t* __restrict__ rank,
                                                     T* __restrict__ dst) {
  const int b = blockIdx.x;
  const FarRec f = rec[b];
  if (f.dense) return;
  const FarDesc a = d[b];
  const int64_t r = rank[b];
  const int64_t nu = r * a.m, nv = r * a.n;
  const T* su = (const T*)a.U;
  const T* sv = (const T*)a.V;
  for (int64_t e = threadIdx.x; e < nu; e += WG) dst[f.uoff + e] = su[e];
  for (int64_t e = threadIdx.x; e < nv; e += WG) dst[f.voff + e] = sv[e];
}

template <class T>
void launch_compact(const FarDesc* d, const FarRec* rec, const int32_t* rank, int64_t nb, T* dst,
                    hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(compact_kernel<T>, dim3((unsigned)nb), dim3(WG), 0, s, d, rec, rank, dst);
  HMX_LAUNCHED();
}

#define HMX_INST(T)                                                                              \
  template void launch_aca<T>(const FarDesc*, const int32_t*, int, int*, const double*,          \
                              const double*, const double*, const double*, int, double, double,  \
                              uint8_t*, int32_t*, int32_t*, int32_t*, double*, int,              \
                              hipStream_t);                                                      \
  template void launch_copy_factors<T>(const FarDesc*, const FarDesc*, const int32_t*,           \
                                       const int32_t*, int, hipStream_t);                        \
  template void launch_compact<T>(const FarDesc*, const FarRec*, const int32_t*, int64_t, T*,    \
                                  hipStream_t);
HMX_INST(double2)
HMX_INST(float2)
#undef HMX_INST

}  // namespace hmx

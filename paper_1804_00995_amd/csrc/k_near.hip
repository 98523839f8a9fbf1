// k_near.hip -- assembly of dense blocks K_b[i, j] = G(x_{t+i}, x_{s+j}) w_{s+j}, column-major
// (element (i, j) at j * m + i), used for the near field and for far blocks stored dense.  With
// the singular correction (Section 5.2) the near-field entries of close pairs also receive their
// correction in the same pass.
#include "hmx_dev.h"
#include "hmx_host.h"
#include "hmx_reg_dev.h"

namespace hmx {

// One workgroup per block; consecutive threads write consecutive entries.  Thread e handles
// entries e, e + WG, ... with (i, j) advanced incrementally (no per-entry division).  REG adds
// the correction (computed in FP64, rounded once into the entry).
template <class T, bool REG>
__global__ void __launch_bounds__(WG) assemble_kernel(
    const int32_t* __restrict__ tb, const int32_t* __restrict__ mm, const int32_t* __restrict__ sb,
    const int32_t* __restrict__ nn, const int64_t* __restrict__ off, const double* __restrict__ X,
    const double* __restrict__ Y, const double* __restrict__ Z, const double* __restrict__ W,
    int kern, const double* __restrict__ kp, T* __restrict__ pool, RegArgs ra) {
  const int blk = blockIdx.x;
  const int t0 = tb[blk], m = mm[blk], s0 = sb[blk], n = nn[blk];
  const double k = kp[t0];  // wavenumber of the block's mesh
  T* K = pool + off[blk];
  const int64_t total = (int64_t)m * n;
  int i = threadIdx.x % m, j = threadIdx.x / m;
  const int di = WG % m, dj = WG / m;
  for (int64_t e = threadIdx.x; e < total; e += WG) {
    double tx = X[t0 + i], ty = Y[t0 + i], tz = Z[t0 + i];
    double sx = X[s0 + j], sy = Y[s0 + j], sz = Z[s0 + j], sw = W[s0 + j];
    T v = eval_entry<T>(kern, k, tx, ty, tz, sx, sy, sz, sw);
    if (REG) {
      const double c = reg_correction(ra, ra.perm[s0 + j], tx, ty, tz, sx, sy, sz, sw);
      if (c != 0.0) {
        double2 vd = to_d2(v);
        vd.x += c;
        v = from_d2<T>(vd);
      }
    }
    K[e] = v;
    i += di;
    j += dj;
    if (i >= m) {
      i -= m;
      j += 1;
    }
  }
}

template <class T>
void launch_assemble(const int32_t* tb, const int32_t* m, const int32_t* sb, const int32_t* n,
                     const int64_t* off, int64_t nblk, const double* X, const double* Y,
                     const double* Z, const double* W, int kern, const double* k, T* pool,
                     const RegArgs* reg, hipStream_t s) {
  if (nblk <= 0) return;
  if (reg) {
    hipLaunchKernelGGL((assemble_kernel<T, true>), dim3((unsigned)nblk), dim3(WG), 0, s, tb, m, sb,
                       n, off, X, Y, Z, W, kern, k, pool, *reg);
  } else {
    hipLaunchKernelGGL((assemble_kernel<T, false>), dim3((unsigned)nblk), dim3(WG), 0, s, tb, m,
                       sb, n, off, X, Y, Z, W, kern, k, pool, RegArgs{});
  }
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

// k_reg.hip -- triangle records of the singular correction (Section 5.2, regularization of the
// kernels): vertices, centroid and squared reach (alpha d_T)^2 per triangle, read by the
// near-field assembly (k_near.hip) for every source point.
#include "hmx_host.h"
#include "hmx_reg_dev.h"

namespace hmx {

// One thread per triangle; the triangle indices were range-checked by the quadrature kernel.
__global__ void __launch_bounds__(WG) tri_geom_kernel(const double* __restrict__ vtx,
                                                      const int32_t* __restrict__ tri, int64_t nt,
                                                      double alpha2, double* __restrict__ tgeo) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t >= nt) return;
  double v[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int64_t a = tri[3 * t + j];
#pragma unroll
    for (int d = 0; d < 3; ++d) v[3 * j + d] = vtx[3 * a + d];
  }
  double d2 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = j == 2 ? 0 : j + 1;
    const double ex = v[3 * k] - v[3 * j], ey = v[3 * k + 1] - v[3 * j + 1],
                 ez = v[3 * k + 2] - v[3 * j + 2];
    d2 = fmax(d2, ex * ex + ey * ey + ez * ez);
  }
  double* g = tgeo + t * TGEO;
#pragma unroll
  for (int e = 0; e < 9; ++e) g[e] = v[e];
#pragma unroll
  for (int d = 0; d < 3; ++d) g[9 + d] = (v[d] + v[3 + d] + v[6 + d]) / 3.0;
  g[12] = alpha2 * d2;
  g[13] = g[14] = g[15] = 0.0;
}

void launch_tri_geom(const double* vtx, const int32_t* tri, int64_t nt, double alpha,
                     double* tgeo, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(tri_geom_kernel, dim3((unsigned)((nt + WG - 1) / WG)), dim3(WG), 0, s, vtx,
                     tri, nt, alpha * alpha, tgeo);
  HMX_LAUNCHED();
}

}  // namespace hmx

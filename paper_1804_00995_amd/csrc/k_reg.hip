// k_reg.hip -- triangle records of the singular correction (Section 5.2, regularization of the
// kernels): vertices, centroid and squared reach (alpha d_T)^2 per triangle, read by the
// near-field assembly (k_near.hip) for every source point.
#include "hmx_host.h"
#include "hmx_reg_dev.h"

namespace hmx {

// One thread per triangle; the triangle indices were range-checked by the quadrature kernel.
// Writes the record described with TGEO (plane frame, edge directions, closeness data).
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
  const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
  const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  const double L = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  double u[3], w[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    n[d] /= nn;
    u[d] = e1[d] / L;
  }
  w[0] = n[1] * u[2] - n[2] * u[1];
  w[1] = n[2] * u[0] - n[0] * u[2];
  w[2] = n[0] * u[1] - n[1] * u[0];
  const double a = e2[0] * u[0] + e2[1] * u[1] + e2[2] * u[2];
  const double b = e2[0] * w[0] + e2[1] * w[1] + e2[2] * w[2];
  double* g = tgeo + t * TGEO;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g[d] = v[d];
    g[3 + d] = u[d];
    g[6 + d] = w[d];
    g[9 + d] = (v[d] + v[3 + d] + v[6 + d]) / 3.0;
    g[13 + d] = n[d];
  }
  g[12] = alpha2 * d2;
  g[16] = L;
  g[17] = a;
  g[18] = b;
  g[19] = 1.0 / (L * b);
  // edges (p0, p1), (p1, p2), (p2, p0) in the plane
  const double pu[3] = {0.0, L, a}, pw[3] = {0.0, 0.0, b};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int j = i == 2 ? 0 : i + 1;
    const double su = pu[j] - pu[i], sw = pw[j] - pw[i];
    const double l2 = su * su + sw * sw, le = sqrt(l2);
    g[20 + 2 * i] = su / le;
    g[21 + 2 * i] = sw / le;
    g[26 + i] = l2;
  }
  g[29] = g[30] = g[31] = 0.0;
}

// iperm[perm[p]] = p: original-to-cluster position map.
__global__ void __launch_bounds__(WG) iperm_kernel(const int32_t* __restrict__ perm, int64_t M,
                                                   int32_t* __restrict__ iperm) {
  const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (p < M) iperm[perm[p]] = (int32_t)p;
}

void launch_iperm(const int32_t* perm, int64_t M, int32_t* iperm, hipStream_t s) {
  if (M <= 0) return;
  hipLaunchKernelGGL(iperm_kernel, dim3((unsigned)((M + WG - 1) / WG)), dim3(WG), 0, s, perm, M,
                     iperm);
  HMX_LAUNCHED();
}

void launch_tri_geom(const double* vtx, const int32_t* tri, int64_t nt, double alpha,
                     double* tgeo, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(tri_geom_kernel, dim3((unsigned)((nt + WG - 1) / WG)), dim3(WG), 0, s, vtx,
                     tri, nt, alpha * alpha, tgeo);
  HMX_LAUNCHED();
}

}  // namespace hmx

// k_quad.hip -- quadrature points and weights of a triangle mesh.
// Compiled without floating-point contraction: the points feed the cluster tree, whose
// comparisons must be reproducible from the same formula evaluated in the written order.
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

// One thread per point m = n_q * t + q:
//   x_m = sum_j lambda_qj * v_{tri[t][j]},  w_m = area(t) * what_q,
//   area(t) = |(b - a) x (c - a)| / 2.
// Out-of-range indices set bit 0 of *err, non-finite coordinates bit 1.
__global__ void __launch_bounds__(WG) quad_kernel(const double* __restrict__ vtx, int64_t nv,
                                                  const int32_t* __restrict__ tri, int64_t nt,
                                                  Rule rule, double* __restrict__ X,
                                                  double* __restrict__ Y, double* __restrict__ Z,
                                                  double* __restrict__ W, int* err) {
  int64_t m = (int64_t)blockIdx.x * WG + threadIdx.x;
  int nq = rule.nq;
  if (m >= nt * nq) return;
  int64_t t = m / nq;
  int q = (int)(m - t * nq);
  int32_t ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
  if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) {
    atomicOr(err, 1);
    X[m] = Y[m] = Z[m] = W[m] = 0.0;
    return;
  }
  const double* a = vtx + 3 * (int64_t)ia;
  const double* b = vtx + 3 * (int64_t)ib;
  const double* c = vtx + 3 * (int64_t)ic;
  double a0 = a[0], a1 = a[1], a2 = a[2], b0 = b[0], b1 = b[1], b2 = b[2], c0 = c[0], c1 = c[1],
         c2 = c[2];
  if (!(isfinite(a0) && isfinite(a1) && isfinite(a2) && isfinite(b0) && isfinite(b1) &&
        isfinite(b2) && isfinite(c0) && isfinite(c1) && isfinite(c2)))
    atomicOr(err, 2);
  double e10 = b0 - a0, e11 = b1 - a1, e12 = b2 - a2;
  double e20 = c0 - a0, e21 = c1 - a1, e22 = c2 - a2;
  double n0 = e11 * e22 - e12 * e21;
  double n1 = e12 * e20 - e10 * e22;
  double n2 = e10 * e21 - e11 * e20;
  double area = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  double l0 = rule.b[q][0], l1 = rule.b[q][1], l2 = rule.b[q][2];
  X[m] = l0 * a0 + l1 * b0 + l2 * c0;
  Y[m] = l0 * a1 + l1 * b1 + l2 * c1;
  Z[m] = l0 * a2 + l1 * b2 + l2 * c2;
  W[m] = area * rule.w[q];
}

void launch_quad(const double* vtx, int64_t nv, const int32_t* tri, int64_t nt, const Rule& rule,
                 double* X, double* Y, double* Z, double* W, int* err, hipStream_t s) {
  int64_t M = nt * rule.nq;
  if (M == 0) return;
  int64_t grid = (M + WG - 1) / WG;
  hipLaunchKernelGGL(quad_kernel, dim3((unsigned)grid), dim3(WG), 0, s, vtx, nv, tri, nt, rule, X,
                     Y, Z, W, err);
  HMX_LAUNCHED();
}

}  // namespace hmx

// k_rwg.hip -- lowest-order Raviart-Thomas (RWG) elements at the quadrature points, for the
// electromagnetic equations of Section 5.5 (EFIE, MFIE, CFIE).
//
// On triangle t the unknown of the edge opposite local vertex j carries
// psi(y) = c_j (y - p_j), c_j = s l_j / (2 A) (s = +-1 the edge's orientation on t), with
// surface divergence 2 c_j.  Per triangle a record of RWG_REC doubles: the vertices p_0..p_2
// (0..8), c_0..c_2 (9..11) and the unit normal (12..14).
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

// one thread per triangle: the record from the vertex coordinates and the edge signs
__global__ void __launch_bounds__(WG) rwg_geom_kernel(const double* __restrict__ vtx,
                                                      const int32_t* __restrict__ tri,
                                                      const int32_t* __restrict__ tsign, int64_t nt,
                                                      double* __restrict__ rec) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t >= nt) return;
  double p[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int d = 0; d < 3; ++d) p[j][d] = vtx[3 * (int64_t)tri[3 * t + j] + d];
  const double e1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
  const double e2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
  const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  const double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  const double area = 0.5 * len;
  double* r = rec + RWG_REC * t;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int d = 0; d < 3; ++d) r[3 * j + d] = p[j][d];
    const double* a = p[(j + 1) % 3];
    const double* b = p[(j + 2) % 3];
    const double l =
        sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]));
    r[9 + j] = tsign[3 * t + j] * l / (2.0 * area);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) r[12 + d] = cr[d] / len;
  r[15] = 0.0;
}

// One thread per quadrature point: u_d = (sum_j x[e_j] psi_j)_d (d < 3) and u_3 = div of it.
template <class T>
__global__ void __launch_bounds__(WG) rwg_interp_kernel(const double* __restrict__ rec,
                                                        const int32_t* __restrict__ tedge,
                                                        int64_t nt, P1Rule rule,
                                                        const T* __restrict__ x, T* __restrict__ u,
                                                        int64_t M) {
  const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (k >= nt * rule.nq) return;
  const int64_t t = k / rule.nq;
  const int q = (int)(k - t * rule.nq);
  const double* r = rec + RWG_REC * t;
  double y[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    y[d] = rule.b[q][0] * r[d] + rule.b[q][1] * r[3 + d] + rule.b[q][2] * r[6 + d];
  double2 s[4] = {};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double2 xe = to_d2(x[tedge[3 * t + j]]);
    const double c = r[9 + j];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double psi = c * (y[d] - r[3 * j + d]);
      s[d].x += psi * xe.x;
      s[d].y += psi * xe.y;
    }
    s[3].x += 2.0 * c * xe.x;
    s[3].y += 2.0 * c * xe.y;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) u[d * M + k] = from_d2<T>(s[d]);
}

// One thread per edge, over its two triangles and their points (fixed order: the + triangle
// first):  y_i = aT sum w psi.ku + aD sum w div(psi) kv + aI sum w psi.u
//               + aN sum w (n x psi).(cp - cm)
// (aT, aD complex; a term is skipped when its coefficient is zero; cm may be null).
template <class T>
__global__ void __launch_bounds__(WG) rwg_project_kernel(const int32_t* __restrict__ einc,
                                                         int64_t ne, const double* __restrict__ rec,
                                                         P1Rule rule, const double* __restrict__ w,
                                                         RwgTerms<T> a, T* __restrict__ yv) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= ne) return;
  double2 sT = {}, sD = {}, sI = {}, sN = {};
  const bool doT = a.aT.x != 0.0 || a.aT.y != 0.0, doD = a.aD.x != 0.0 || a.aD.y != 0.0;
  const bool doI = a.aI != 0.0, doN = a.aN != 0.0;
  for (int side = 0; side < 2; ++side) {
    const int32_t inc = einc[2 * e + side];
    const int64_t t = inc / 3;
    const int j = inc - 3 * (int)t;
    const double* r = rec + RWG_REC * t;
    const double c = r[9 + j];
    for (int q = 0; q < rule.nq; ++q) {
      const int64_t k = t * rule.nq + q;
      double psi[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        psi[d] = c * (rule.b[q][0] * r[d] + rule.b[q][1] * r[3 + d] + rule.b[q][2] * r[6 + d] -
                      r[3 * j + d]);
      const double wk = w[k];
      if (doT) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double2 v = to_d2(a.ku[d][k]);
          sT.x += wk * psi[d] * v.x;
          sT.y += wk * psi[d] * v.y;
        }
      }
      if (doD) {
        const double2 v = to_d2(a.kv[k]);
        sD.x += wk * 2.0 * c * v.x;
        sD.y += wk * 2.0 * c * v.y;
      }
      if (doI) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double2 v = to_d2(a.u[d][k]);
          sI.x += wk * psi[d] * v.x;
          sI.y += wk * psi[d] * v.y;
        }
      }
      if (doN) {
        const double np[3] = {r[13] * psi[2] - r[14] * psi[1], r[14] * psi[0] - r[12] * psi[2],
                              r[12] * psi[1] - r[13] * psi[0]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double2 v = to_d2(a.cp[d][k]);
          if (a.cm[d]) {
            const double2 m = to_d2(a.cm[d][k]);
            v.x -= m.x;
            v.y -= m.y;
          }
          sN.x += wk * np[d] * v.x;
          sN.y += wk * np[d] * v.y;
        }
      }
    }
  }
  double2 o;
  o.x = a.aT.x * sT.x - a.aT.y * sT.y + a.aD.x * sD.x - a.aD.y * sD.y + a.aI * sI.x + a.aN * sN.x;
  o.y = a.aT.x * sT.y + a.aT.y * sT.x + a.aD.x * sD.y + a.aD.y * sD.x + a.aI * sI.y + a.aN * sN.y;
  yv[e] = from_d2<T>(o);
}

static unsigned nblk(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

void launch_rwg_geom(const double* vtx, const int32_t* tri, const int32_t* tsign, int64_t nt,
                     double* rec, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(rwg_geom_kernel, dim3(nblk(nt)), dim3(WG), 0, s, vtx, tri, tsign, nt, rec);
  HMX_LAUNCHED();
}

template <class T>
void launch_rwg_interp(const double* rec, const int32_t* tedge, int64_t nt, const P1Rule& r,
                       const T* x, T* u, hipStream_t s) {
  if (nt <= 0) return;
  const int64_t M = nt * r.nq;
  hipLaunchKernelGGL(rwg_interp_kernel<T>, dim3(nblk(M)), dim3(WG), 0, s, rec, tedge, nt, r, x, u, M);
  HMX_LAUNCHED();
}

template <class T>
void launch_rwg_project(const int32_t* einc, int64_t ne, const double* rec, const P1Rule& r,
                        const double* w, const RwgTerms<T>& a, T* y, hipStream_t s) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(rwg_project_kernel<T>, dim3(nblk(ne)), dim3(WG), 0, s, einc, ne, rec, r, w, a, y);
  HMX_LAUNCHED();
}

#define HMX_INST(T)                                                                             \
  template void launch_rwg_interp<T>(const double*, const int32_t*, int64_t, const P1Rule&,      \
                                     const T*, T*, hipStream_t);                                \
  template void launch_rwg_project<T>(const int32_t*, int64_t, const double*, const P1Rule&,     \
                                      const double*, const RwgTerms<T>&, T*, hipStream_t);
HMX_INST(double2)
HMX_INST(float2)
#undef HMX_INST

}  // namespace hmx

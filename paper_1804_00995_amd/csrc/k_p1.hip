// k_p1.hip -- P1 finite elements at the quadrature points (eq. (BEM): the basis functions
// evaluated at the points, Phi[n_q t + q, v] = lambda_v(point q of triangle t)) and the vector
// kernels of the GMRES solver of Galerkin systems.
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

// xp[n_q t + q] = sum_j bary[q][j] xv[tri[t][j]]: one thread per point.
template <class T>
__global__ void __launch_bounds__(WG) p1_interp_kernel(const int32_t* __restrict__ tri, int64_t nt,
                                                       P1Rule rule, const T* __restrict__ xv,
                                                       T* __restrict__ xp) {
  const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (k >= nt * rule.nq) return;
  const int64_t t = k / rule.nq;
  const int q = (int)(k - t * rule.nq);
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double2 v = to_d2(xv[tri[3 * t + j]]);
    s.x += rule.b[q][j] * v.x;
    s.y += rule.b[q][j] * v.y;
  }
  xp[k] = from_d2<T>(s);
}

// yv[v] = sum over the incidences (t, j) of vertex v (inc[ptr[v] .. ptr[v + 1]) = 3 t + j, in
// increasing t) of sum_q bary[q][j] w[n_q t + q] zp[n_q t + q]: Phi^T W z, one thread per
// vertex, in a fixed order (no atomics).
template <class T>
__global__ void __launch_bounds__(WG) p1_project_kernel(const int64_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ inc, int64_t nv,
                                                        P1Rule rule, const double* __restrict__ w,
                                                        const T* __restrict__ zp,
                                                        T* __restrict__ yv) {
  const int64_t v = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (v >= nv) return;
  double2 s = make_double2(0.0, 0.0);
  for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
    const int64_t t = inc[e] / 3;
    const int j = inc[e] - 3 * (int)t;
    for (int q = 0; q < rule.nq; ++q) {
      const int64_t k = t * rule.nq + q;
      const double c = rule.b[q][j] * w[k];
      const double2 z = to_d2(zp[k]);
      s.x += c * z.x;
      s.y += c * z.y;
    }
  }
  yv[v] = from_d2<T>(s);
}

// Batched dot products d[c] = V_c^H w (c < nc, V column-major with leading dimension ld) in FP64:
// grid (chunks, nc); each workgroup sums one column over one chunk of MDOT_CHUNK elements.
constexpr int MDOT_CHUNK = 8 * WG;

template <class T>
__global__ void __launch_bounds__(WG) mdot_kernel(const T* __restrict__ V, int64_t ld,
                                                  const T* __restrict__ w, int64_t n,
                                                  double2* __restrict__ partial) {
  __shared__ double sh[2 * NWAVE + 2];
  const int c = blockIdx.y;
  const T* vc = V + (int64_t)c * ld;
  const int64_t e0 = (int64_t)blockIdx.x * MDOT_CHUNK;
  const int64_t e1 = min(e0 + (int64_t)MDOT_CHUNK, n);
  double re = 0.0, im = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += WG) {
    const double2 a = to_d2(vc[e]), b = to_d2(w[e]);
    re += a.x * b.x + a.y * b.y;  // conj(a) b
    im += a.x * b.y - a.y * b.x;
  }
  double v[2] = {re, im};
  block_sum<2, WG>(v, sh);
  if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = make_double2(v[0], v[1]);
}

// d[c] = sum of the chunk partial sums of column c (one thread per column, fixed order).
__global__ void mdot_reduce_kernel(const double2* __restrict__ partial, int nchunk, int nc,
                                   double2* __restrict__ d) {
  const int c = blockIdx.x * WG + threadIdx.x;
  if (c >= nc) return;
  double2 s = make_double2(0.0, 0.0);
  for (int b = 0; b < nchunk; ++b) {
    s.x += partial[(int64_t)c * nchunk + b].x;
    s.y += partial[(int64_t)c * nchunk + b].y;
  }
  d[c] = s;
}

// w += sign * sum_{c < nc} V_c h[c] (h in FP64, on the device).
template <class T>
__global__ void __launch_bounds__(WG) gemv_update_kernel(const T* __restrict__ V, int64_t ld,
                                                         const double2* __restrict__ h, int nc,
                                                         double sign, T* __restrict__ w,
                                                         int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n) return;
  double2 s = to_d2(w[e]);
  for (int c = 0; c < nc; ++c) {
    const double2 a = to_d2(V[(int64_t)c * ld + e]), b = h[c];
    s.x += sign * (a.x * b.x - a.y * b.y);
    s.y += sign * (a.x * b.y + a.y * b.x);
  }
  w[e] = from_d2<T>(s);
}

// y = a * x (a real), or y = b - x when sub != 0.
template <class T>
__global__ void __launch_bounds__(WG) vec_kernel(const T* __restrict__ x, const T* __restrict__ b,
                                                 double a, int sub, T* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n) return;
  const double2 v = to_d2(x[e]);
  if (sub) {
    const double2 c = to_d2(b[e]);
    y[e] = from_d2<T>(make_double2(c.x - v.x, c.y - v.y));
  } else {
    y[e] = from_d2<T>(make_double2(a * v.x, a * v.y));
  }
}

static unsigned nblk(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

template <class T>
void launch_p1_interp(const int32_t* tri, int64_t nt, const P1Rule& r, const T* xv, T* xp,
                      hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(p1_interp_kernel<T>, dim3(nblk(nt * r.nq)), dim3(WG), 0, s, tri, nt, r, xv,
                     xp);
  HMX_LAUNCHED();
}

template <class T>
void launch_p1_project(const int64_t* ptr, const int32_t* inc, int64_t nv, const P1Rule& r,
                       const double* w, const T* zp, T* yv, hipStream_t s) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(p1_project_kernel<T>, dim3(nblk(nv)), dim3(WG), 0, s, ptr, inc, nv, r, w, zp,
                     yv);
  HMX_LAUNCHED();
}

int mdot_chunks(int64_t n) { return (int)((n + MDOT_CHUNK - 1) / MDOT_CHUNK); }

template <class T>
void launch_mdot(const T* V, int64_t ld, int nc, const T* w, int64_t n, double2* partial,
                 double2* d, hipStream_t s) {
  const int nch = mdot_chunks(n);
  hipLaunchKernelGGL(mdot_kernel<T>, dim3((unsigned)nch, (unsigned)nc), dim3(WG), 0, s, V, ld, w, n,
                     partial);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(mdot_reduce_kernel, dim3(nblk(nc)), dim3(WG), 0, s, partial, nch, nc, d);
  HMX_LAUNCHED();
}

template <class T>
void launch_gemv_update(const T* V, int64_t ld, const double2* h, int nc, double sign, T* w,
                        int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(gemv_update_kernel<T>, dim3(nblk(n)), dim3(WG), 0, s, V, ld, h, nc, sign, w,
                     n);
  HMX_LAUNCHED();
}

template <class T>
void launch_vec(const T* x, const T* b, double a, int sub, T* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(vec_kernel<T>, dim3(nblk(n)), dim3(WG), 0, s, x, b, a, sub, y, n);
  HMX_LAUNCHED();
}

#define HMX_INST(T)                                                                             \
  template void launch_p1_interp<T>(const int32_t*, int64_t, const P1Rule&, const T*, T*,        \
                                    hipStream_t);                                               \
  template void launch_p1_project<T>(const int64_t*, const int32_t*, int64_t, const P1Rule&,     \
                                     const double*, const T*, T*, hipStream_t);                 \
  template void launch_mdot<T>(const T*, int64_t, int, const T*, int64_t, double2*, double2*,    \
                               hipStream_t);                                                    \
  template void launch_gemv_update<T>(const T*, int64_t, const double2*, int, double, T*,        \
                                      int64_t, hipStream_t);                                    \
  template void launch_vec<T>(const T*, const T*, double, int, T*, int64_t, hipStream_t);
HMX_INST(double2)
HMX_INST(float2)
#undef HMX_INST

}  // namespace hmx

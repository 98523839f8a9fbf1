// hmx_dev.h -- device-side building blocks shared by the HIP kernels of libhmx.
//
// Complex numbers are interleaved pairs (double2 for c128, float2 for c64).  Wavefronts are 64
// lanes wide (CDNA); workgroups used by the kernels are 256 threads = 4 wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Address-space qualifiers of device pointers whose space the compiler cannot infer (addresses
// read from memory): global (1) and LDS (3).  They matter only to device code generation, so the
// host pass of the same source, which checks kernel bodies without generating them, sees plain
// pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define HMX_GLOBAL __attribute__((address_space(1)))
#define HMX_LDS __attribute__((address_space(3)))
#else
#define HMX_GLOBAL
#define HMX_LDS
#endif

namespace hmx {

constexpr int WG = 256;
constexpr int WAVE = 64;
constexpr int NWAVE = WG / WAVE;
constexpr double INV4PI = 0.079577471545947667884441881686257181;  // 1 / (4 pi)
constexpr double TWO_PI = 6.283185307179586476925286766559005768;

enum KernelId : int32_t {
  K_LAPLACE = 0,
  K_HELMHOLTZ = 1,
  K_GRADY_X = 2,  // dG/dy_j, j = kern - K_GRADY_X
  K_GRADY_Y = 3,
  K_GRADY_Z = 4,
  K_POLY2 = 99
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a += b * c
__device__ __forceinline__ void cfma(double2& a, double2 b, double2 c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(b.y, c.x, a.y);
}
__device__ __forceinline__ void cfma(float2& a, float2 b, float2 c) {
  a.x = fmaf(b.x, c.x, a.x);
  a.x = fmaf(-b.y, c.y, a.x);
  a.y = fmaf(b.x, c.y, a.y);
  a.y = fmaf(b.y, c.x, a.y);
}
// a -= b * c
__device__ __forceinline__ void cfms(double2& a, double2 b, double2 c) {
  a.x = fma(-b.x, c.x, a.x);
  a.x = fma(b.y, c.y, a.x);
  a.y = fma(-b.x, c.y, a.y);
  a.y = fma(-b.y, c.x, a.y);
}

// r = sqrt(r2) and y = 1 / r for r2 > 0 without the square-root and division sequences: the
// hardware reciprocal square root y0, one third-order Newton step y = y0 (1 + e/2 + 3 e^2/8)
// with e = 1 - r2 y0^2 (the relative error is cubed, so a start good to about 2^-18 ends at
// rounding level), then r0 = r2 y and one Newton step of the square root with the exact
// residual r2 - r0^2 (an fma), which rounds r like the IEEE square root except in rare near-ties.
// Outside [2^-900, 2^900] (never reached by surface meshes of sane coordinates) the IEEE
// square root and division.
__device__ __forceinline__ void dist_inv(double r2, double& r, double& y) {
  if (r2 < 0x1p-900 || r2 > 0x1p900) {
    r = sqrt(r2);
    y = 1.0 / r;
    return;
  }
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double e = fma(-(r2 * y0), y0, 1.0);
  y = fma(y0 * e, fma(0.375, e, 0.5), y0);
  const double r0 = r2 * y;
  r = fma(0.5 * y, fma(-r0, r0, r2), r0);
}

// Green kernel between a target x and a source y, FP64 throughout:
// G = e^{i k r} / (4 pi r), r = |x - y|; 0 when r == 0; Laplace is the real 1/(4 pi r);
// POLY2 is the test-only separable kernel (1 + x.y)^2.
__device__ __forceinline__ double2 green64(int kern, double k, double xx, double xy, double xz,
                                           double yx, double yy, double yz) {
  if (kern == K_POLY2) {
    double d = 1.0 + (xx * yx + xy * yy + xz * yz);
    return make_double2(d * d, 0.0);
  }
  double dx = xx - yx, dy = xy - yy, dz = xz - yz;
  double r2 = dx * dx + dy * dy + dz * dz;
  if (r2 == 0.0) return make_double2(0.0, 0.0);
  double r, ir;
  dist_inv(r2, r, ir);
  if (kern >= K_GRADY_X && kern <= K_GRADY_Z) {
    // dG/dy_j = e^{ikr} (ikr - 1) (y_j - x_j) / (4 pi r^3)
    const double d = kern == K_GRADY_X ? -dx : (kern == K_GRADY_Y ? -dy : -dz);
    const double f = d * INV4PI * (ir * ir * ir), kr = k * r;
    double s, c;
    sincos(kr, &s, &c);
    return make_double2(f * (-c - kr * s), f * (kr * c - s));
  }
  double inv = INV4PI * ir;
  if (kern == K_LAPLACE) return make_double2(inv, 0.0);
  double s, c;
  sincos(k * r, &s, &c);
  return make_double2(c * inv, s * inv);
}

// Mixed-precision Green kernel: distance and phase k r in FP64 (the phase reduced to
// [-pi, pi] in FP64), sin/cos and the 1/(4 pi r) scaling in FP32.
__device__ __forceinline__ float2 green32(int kern, double k, double xx, double xy, double xz,
                                          double yx, double yy, double yz) {
  if (kern == K_POLY2) {
    double d = 1.0 + (xx * yx + xy * yy + xz * yz);
    return make_float2((float)(d * d), 0.0f);
  }
  double dx = xx - yx, dy = xy - yy, dz = xz - yz;
  double r2 = dx * dx + dy * dy + dz * dz;
  if (r2 == 0.0) return make_float2(0.0f, 0.0f);
  double r, ir;
  dist_inv(r2, r, ir);
  if (kern >= K_GRADY_X && kern <= K_GRADY_Z) {
    const double d = kern == K_GRADY_X ? -dx : (kern == K_GRADY_Y ? -dy : -dz);
    const float f = (float)(d * INV4PI * (ir * ir * ir)), kr = (float)(k * r);
    double ph = k * r;
    ph = ph - TWO_PI * rint(ph * (1.0 / TWO_PI));
    float s, c;
    __sincosf((float)ph, &s, &c);
    return make_float2(f * (-c - kr * s), f * (kr * c - s));
  }
  float inv = (float)(INV4PI * ir);
  if (kern == K_LAPLACE) return make_float2(inv, 0.0f);
  double ph = k * r;
  ph = ph - TWO_PI * rint(ph * (1.0 / TWO_PI));
  float s, c;
  __sincosf((float)ph, &s, &c);
  return make_float2(c * inv, s * inv);
}

// ----------------------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// (value, index) argmax with the lowest index winning ties.
__device__ __forceinline__ void amax_merge(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}
__device__ __forceinline__ void wave_amax(double& v, int& i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double v2 = __shfl_xor(v, o, WAVE);
    int i2 = __shfl_xor(i, o, WAVE);
    amax_merge(v, i, v2, i2);
  }
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Workgroup-wide argmax over NT threads; every thread receives the result.
// `sv`, `si` are LDS scratch of NT / 64 entries.
template <int NT = WG>
__device__ __forceinline__ void block_amax(double& v, int& i, double* sv, int* si) {
  constexpr int NW = NT / WAVE;
  wave_amax(v, i);
  int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) amax_merge(v, i, sv[q], si[q]);
}

template <int NT = WG>
__device__ __forceinline__ int block_min(int v, int* s) {
  constexpr int NW = NT / WAVE;
  v = wave_min(v);
  int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) s[w] = v;
  __syncthreads();
  int r = s[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) r = min(r, s[q]);
  return r;
}

// Sum of N doubles per thread over NT threads, in a fixed order (deterministic): wavefront
// sums, then thread q adds the NT / 64 partials of value q, then every thread reads the N sums.
// `s` is LDS scratch of N * (NT / 64 + 1) doubles; N <= NT.
template <int N, int NT = WG>
__device__ __forceinline__ void block_sum(double* v, double* s) {
  constexpr int NW = NT / WAVE;
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) s[q * NW + w] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int q = threadIdx.x;
    double a = s[q * NW];
    for (int p = 1; p < NW; ++p) a += s[q * NW + p];
    s[N * NW + q] = a;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = s[N * NW + q];
}

// Exclusive scan of one int per thread over the workgroup; returns the thread's prefix and
// writes the total to *total.  `s` is LDS scratch of NWAVE ints.
__device__ __forceinline__ int block_excl_scan(int v, int* s, int* total) {
  int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  int x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == WAVE - 1) s[w] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NWAVE; ++q) {
    if (q < w) base += s[q];
    tot += s[q];
  }
  *total = tot;
  return base + x - v;
}

// Order-preserving map of doubles to unsigned 64-bit keys (for atomic min/max and sorting).
__device__ __forceinline__ unsigned long long dkey(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// ------------------------------------------------------------------ typed entry helpers
// Entry K(i, j) = G(x_i, x_j) w_j in the storage precision T (double2: FP64 throughout;
// float2: FP64 distance and phase, FP32 values).
template <class T>
__device__ __forceinline__ T eval_entry(int kern, double k, double tx, double ty, double tz,
                                        double sx, double sy, double sz, double sw);
template <>
__device__ __forceinline__ double2 eval_entry<double2>(int kern, double k, double tx, double ty,
                                                       double tz, double sx, double sy, double sz,
                                                       double sw) {
  double2 g = green64(kern, k, tx, ty, tz, sx, sy, sz);
  return make_double2(g.x * sw, g.y * sw);
}
template <>
__device__ __forceinline__ float2 eval_entry<float2>(int kern, double k, double tx, double ty,
                                                     double tz, double sx, double sy, double sz,
                                                     double sw) {
  float2 g = green32(kern, k, tx, ty, tz, sx, sy, sz);
  float w = (float)sw;
  return make_float2(g.x * w, g.y * w);
}

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <class T> __device__ __forceinline__ T from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double abs2(double2 v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double abs2(float2 v) {
  double x = v.x, y = v.y;
  return x * x + y * y;
}
__device__ __forceinline__ void cfms(float2& a, float2 b, float2 c) {
  a.x = fmaf(-b.x, c.x, a.x);
  a.x = fmaf(b.y, c.y, a.x);
  a.y = fmaf(-b.x, c.y, a.y);
  a.y = fmaf(-b.y, c.x, a.y);
}
template <class T> __device__ __forceinline__ T czero();
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.0f, 0.0f); }

}  // namespace hmx

namespace hmx {
// Value of lane `lane` (wave-uniform) broadcast to the whole wavefront.
__device__ __forceinline__ double readlane(double x, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double2 readlane(double2 v, int lane) {
  return make_double2(readlane(v.x, lane), readlane(v.y, lane));
}
__device__ __forceinline__ float2 readlane(float2 v, int lane) {
  return make_float2(readlane(v.x, lane), readlane(v.y, lane));
}
}  // namespace hmx

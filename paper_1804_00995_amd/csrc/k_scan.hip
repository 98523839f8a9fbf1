// k_scan.hip -- device utilities used by the build: exclusive prefix sums and fills.
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = WG * SCAN_ITEMS;

__device__ __forceinline__ long long block_excl_scan_ll(long long v, long long* s, long long* total) {
  int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  long long x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    long long y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == WAVE - 1) s[w] = x;
  __syncthreads();
  long long base = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NWAVE; ++q) {
    if (q < w) base += s[q];
    tot += s[q];
  }
  *total = tot;
  return base + x - v;
}

__global__ void __launch_bounds__(WG) scan_sums_kernel(const int64_t* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ bsum) {
  __shared__ long long s[NWAVE];
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  long long acc = 0;
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    int64_t i = base + (int64_t)q * WG + threadIdx.x;
    if (i < n) acc += in[i];
  }
  long long tot;
  block_excl_scan_ll(acc, s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(WG) scan_offsets_kernel(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ long long s[NWAVE];
  long long run = 0;
  for (int64_t c = 0; c < nb; c += WG) {
    int64_t i = c + threadIdx.x;
    long long v = i < nb ? bsum[i] : 0;
    long long tot;
    long long pre = block_excl_scan_ll(v, s, &tot);
    if (i < nb) bsum[i] = run + pre;
    run += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = run;
}

__global__ void __launch_bounds__(WG) scan_apply_kernel(const int64_t* __restrict__ in, int64_t n,
                                                        const int64_t* __restrict__ boff,
                                                        int64_t nb, int64_t* __restrict__ out) {
  __shared__ long long s[NWAVE];
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  long long v[SCAN_ITEMS];
  long long acc = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    int64_t i = base + q;
    v[q] = i < n ? in[i] : 0;
    acc += v[q];
  }
  long long tot;
  long long pre = block_excl_scan_ll(acc, s, &tot) + boff[blockIdx.x];
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    int64_t i = base + q;
    if (i < n) out[i] = pre;
    pre += v[q];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = boff[nb];
}

int64_t scan_work_len(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

void scan_excl_i64_work(const int64_t* in, int64_t* out, int64_t n, int64_t* bsum,
                        hipStream_t s) {
  if (n == 0) {
    fill_i64(out, 0, 1, s);
    return;
  }
  int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(WG), 0, s, in, n, bsum);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(scan_offsets_kernel, dim3(1), dim3(WG), 0, s, bsum, nb);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(WG), 0, s, in, n, bsum, nb, out);
  HMX_LAUNCHED();
}

void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  DevBuf<int64_t> bsum(scan_work_len(n));
  scan_excl_i64_work(in, out, n, bsum.p, s);
  HMX_HIP(hipStreamSynchronize(s));  // bsum is freed on return
}

template <class T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class T>
static void fill_any(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, p, v, n);
  HMX_LAUNCHED();
}
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { fill_any(p, v, n, s); }
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) { fill_any(p, v, n, s); }
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { fill_any(p, v, n, s); }
void fill_f64(double* p, double v, int64_t n, hipStream_t s) { fill_any(p, v, n, s); }

__global__ void iota_kernel(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}
void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, p, n);
  HMX_LAUNCHED();
}

}  // namespace hmx

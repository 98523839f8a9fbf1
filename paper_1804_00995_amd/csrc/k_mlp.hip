// k_mlp.hip -- block-rank MLP: features of far blocks, inference, and training kernels.
//
// The network maps the standardized features of a far block
//   [log2 m, log2 n, ln(dist / max diam), k max diam / (2 pi)]
// through 4 -> 64 -> 64 -> 1 with ReLU activations to a prediction of ln(1 + rank).  The
// parameter vector is W1 (64 x 4) | b1 (64) | W2 (64 x 64) | b2 (64) | W3 (64) | b3 (1), FP32.
//
// Training step on a minibatch of B samples (mean squared error):
//   mlp_fwdbwd: one thread per sample: activations, residual and the back-propagated errors
//               dL/dz2, dL/dz1, stored per sample (structure of arrays, sample index fastest);
//   mlp_grad:   one wavefront per parameter: its gradient summed over the batch in a fixed order
//               (FP64 accumulation), so the result does not depend on scheduling;
//   mlp_adam:   one thread per parameter: bias-corrected Adam update.
#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {

constexpr int NI = MLP_IN, NH = MLP_H;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH;
static_assert(OB3 + 1 == MLP_NPARAMS, "parameter layout");

__global__ void __launch_bounds__(WG) mlp_features_kernel(
    const int2* __restrict__ pairs, int64_t n, const int32_t* __restrict__ nbegin,
    const int32_t* __restrict__ nend, const double* __restrict__ box,
    const double* __restrict__ kp, float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const int2 p = pairs[i];
  const double* a = box + 6 * (int64_t)p.x;
  const double* b = box + 6 * (int64_t)p.y;
  double da = 0.0, db = 0.0, dist = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double ea = a[3 + d] - a[d], eb = b[3 + d] - b[d];
    da += ea * ea;
    db += eb * eb;
    double g = 0.0;
    if (b[d] - a[3 + d] > g) g = b[d] - a[3 + d];
    if (a[d] - b[3 + d] > g) g = a[d] - b[3 + d];
    dist += g * g;
  }
  const double dmax = fmax(fmax(sqrt(da), sqrt(db)), 1e-12);
  const double m = (double)(nend[p.x] - nbegin[p.x]), nn = (double)(nend[p.y] - nbegin[p.y]);
  feat[4 * i + 0] = (float)log2(m);
  feat[4 * i + 1] = (float)log2(nn);
  feat[4 * i + 2] = (float)log(fmax(sqrt(dist), 1e-12) / dmax);
  feat[4 * i + 3] = (float)(kp[nbegin[p.x]] * dmax / TWO_PI);  // k of the block's mesh
}

void launch_mlp_features(const int2* pairs, int64_t n, const int32_t* nbegin, const int32_t* nend,
                         const double* box, const double* kp, float* feat, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s,
                     pairs, n, nbegin, nend, box, kp, feat);
  HMX_LAUNCHED();
}

// Inference: one thread per sample, parameters in LDS.  `norm` = mean[4], std[4].
__global__ void __launch_bounds__(WG) mlp_predict_kernel(const float* __restrict__ theta,
                                                         const float* __restrict__ norm,
                                                         const float* __restrict__ feat, int64_t n,
                                                         float* __restrict__ out) {
  __shared__ float w[MLP_NPARAMS];
  __shared__ float nm[8];
  for (int q = threadIdx.x; q < MLP_NPARAMS; q += WG) w[q] = theta[q];
  if (threadIdx.x < 8) nm[threadIdx.x] = norm[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  float x[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) x[c] = (feat[4 * i + c] - nm[c]) / nm[4 + c];
  float h1[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float z = w[OB1 + j];
#pragma unroll
    for (int c = 0; c < NI; ++c) z = fmaf(w[OW1 + j * NI + c], x[c], z);
    h1[j] = fmaxf(z, 0.0f);
  }
  float o = w[OB3];
  for (int j = 0; j < NH; ++j) {
    float z = w[OB2 + j];
#pragma unroll
    for (int c = 0; c < NH; ++c) z = fmaf(w[OW2 + j * NH + c], h1[c], z);
    o = fmaf(w[OW3 + j], fmaxf(z, 0.0f), o);
  }
  out[i] = o;
}

void launch_mlp_predict(const float* theta, const float* norm, const float* feat, int64_t n,
                        float* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, theta,
                     norm, feat, n, out);
  HMX_LAUNCHED();
}

// Per-sample forward and backward pass over samples [b0, b0 + B) of (X, y); X standardized.
// Cache layout (floats, sample fastest): x[4][B] h1[64][B] h2[64][B] dz1[64][B] dz2[64][B]
// do[B] r2[B].
__global__ void __launch_bounds__(WG) mlp_fwdbwd_kernel(const float* __restrict__ theta,
                                                        const float* __restrict__ X,
                                                        const float* __restrict__ y, int64_t b0,
                                                        int B, float* __restrict__ cache) {
  __shared__ float w[MLP_NPARAMS];
  for (int q = threadIdx.x; q < MLP_NPARAMS; q += WG) w[q] = theta[q];
  __syncthreads();
  const int s = blockIdx.x * WG + threadIdx.x;
  if (s >= B) return;
  float* cx = cache;
  float* ch1 = cx + (int64_t)NI * B;
  float* ch2 = ch1 + (int64_t)NH * B;
  float* cd1 = ch2 + (int64_t)NH * B;
  float* cd2 = cd1 + (int64_t)NH * B;
  float* cdo = cd2 + (int64_t)NH * B;
  float* cr2 = cdo + B;
  const int64_t g = b0 + s;
  float x[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    x[c] = X[4 * g + c];
    cx[(int64_t)c * B + s] = x[c];
  }
  float z1[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float z = w[OB1 + j];
#pragma unroll
    for (int c = 0; c < NI; ++c) z = fmaf(w[OW1 + j * NI + c], x[c], z);
    z1[j] = z;
    ch1[(int64_t)j * B + s] = fmaxf(z, 0.0f);
  }
  float o = w[OB3];
  float z2[NH];  // pre-activations, then dL/dz2 in place
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float z = w[OB2 + j];
#pragma unroll
    for (int c = 0; c < NH; ++c) z = fmaf(w[OW2 + j * NH + c], fmaxf(z1[c], 0.0f), z);
    z2[j] = z;
    const float h2 = fmaxf(z, 0.0f);
    ch2[(int64_t)j * B + s] = h2;
    o = fmaf(w[OW3 + j], h2, o);
  }
  const float r = o - y[g];
  const float dout = 2.0f * r / (float)B;
  cdo[s] = dout;
  cr2[s] = r * r;
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    z2[j] = z2[j] > 0.0f ? dout * w[OW3 + j] : 0.0f;
    cd2[(int64_t)j * B + s] = z2[j];
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    float d = 0.0f;
#pragma unroll
    for (int j = 0; j < NH; ++j) d = fmaf(z2[j], w[OW2 + j * NH + i], d);
    cd1[(int64_t)i * B + s] = z1[i] > 0.0f ? d : 0.0f;
  }
}

// Gradient of parameter p (p < MLP_NPARAMS) summed over the batch; p == MLP_NPARAMS gives the
// batch loss (1/B) sum r^2.  One wavefront per output value, fixed summation order.
__global__ void __launch_bounds__(WG) mlp_grad_kernel(const float* __restrict__ cache, int B,
                                                      float* __restrict__ grad) {
  const int p = blockIdx.x * NWAVE + threadIdx.x / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (p > MLP_NPARAMS) return;
  const float* cx = cache;
  const float* ch1 = cx + (int64_t)NI * B;
  const float* ch2 = ch1 + (int64_t)NH * B;
  const float* cd1 = ch2 + (int64_t)NH * B;
  const float* cd2 = cd1 + (int64_t)NH * B;
  const float* cdo = cd2 + (int64_t)NH * B;
  const float* cr2 = cdo + B;
  const float* a = nullptr;  // first factor
  const float* b = nullptr;  // second factor (nullptr: 1)
  double scale = 1.0;
  if (p < OB1) {
    const int j = (p - OW1) / NI, c = (p - OW1) % NI;
    a = cd1 + (int64_t)j * B;
    b = cx + (int64_t)c * B;
  } else if (p < OW2) {
    a = cd1 + (int64_t)(p - OB1) * B;
  } else if (p < OB2) {
    const int j = (p - OW2) / NH, i = (p - OW2) % NH;
    a = cd2 + (int64_t)j * B;
    b = ch1 + (int64_t)i * B;
  } else if (p < OW3) {
    a = cd2 + (int64_t)(p - OB2) * B;
  } else if (p < OB3) {
    a = cdo;
    b = ch2 + (int64_t)(p - OW3) * B;
  } else if (p == OB3) {
    a = cdo;
  } else {
    a = cr2;
    scale = 1.0 / (double)B;
  }
  double acc = 0.0;
  for (int s = lane; s < B; s += WAVE) acc += b ? (double)a[s] * (double)b[s] : (double)a[s];
  acc = wave_sum(acc);
  if (lane == 0) grad[p] = (float)(acc * scale);
}

__global__ void mlp_adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                float* __restrict__ m, float* __restrict__ v, float lr, float c1,
                                float c2) {
  const int p = blockIdx.x * WG + threadIdx.x;
  if (p >= MLP_NPARAMS) return;
  const float g = grad[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

size_t mlp_cache_floats(int B) { return (size_t)(NI + 4 * NH + 2) * (size_t)B; }

void launch_mlp_grad(const float* theta, const float* X, const float* y, int64_t b0, int B,
                     float* cache, float* grad, hipStream_t s) {
  hipLaunchKernelGGL(mlp_fwdbwd_kernel, dim3((B + WG - 1) / WG), dim3(WG), 0, s, theta, X, y, b0,
                     B, cache);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((MLP_NPARAMS + 1 + NWAVE - 1) / NWAVE), dim3(WG), 0, s,
                     cache, B, grad);
  HMX_LAUNCHED();
}

void launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr,
                     hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAMS + WG - 1) / WG), dim3(WG), 0, s, theta,
                     grad, m, v, lr, c1, c2);
  HMX_LAUNCHED();
}

}  // namespace hmx

// k_mlp.hip -- block-rank MLP: features of far blocks, inference, and training kernels.
//
// The network maps the standardized features of a far block
//   [log2 m, log2 n, ln(dist / max diam), k max diam / (2 pi)]
// through 4 -> 64 -> 64 -> 1 with ReLU activations to a prediction of ln(1 + rank).  The
// parameter vector is W1 (64 x 4) | b1 (64) | W2 (64 x 64) | b2 (64) | W3 (64) | b3 (1), FP32.
//
// Training step on a minibatch of B samples (mean squared error):
//   mlp_tile_grad: one wavefront per 16 samples: forward and backward pass with the 64 x 64
//                  layer on the FP32 matrix cores, and the tile's partial gradient;
//   mlp_reduce:    one thread per parameter: the tiles' partials summed in a fixed order (FP64),
//                  so the result does not depend on scheduling;
//   mlp_adam:      one thread per parameter: bias-corrected Adam update.
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

// ------------------------------------------------------------------------------ training
// Minibatch gradient of the mean squared error over samples [b0, b0 + B) of (X, y), X
// standardized.  One wavefront per tile of 16 samples (a 4096-sample batch is 256 wavefronts,
// one per CU); lane l works on sample s = l % 16 of the tile and on the 16 hidden units
//   u(t, g) = 16 (t / 4) + 4 g + (t % 4),  t = 0..15,  g = l / 16,
// in both hidden layers.  With that assignment the 64 x 64 layer and its transpose run on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32: A 16 x 4 from lane i + 16 k, B 4 x 16 from lane
// j + 16 k, D 16 x 16 in lane j + 16 (i / 4), element i % 4) with every operand already in the
// lane that supplies it:
//   Z2^T = W2 H1^T      (A = W2 rows, B = the lane's own h1[t], k-step t)
//   dH1^T = W2^T dZ2^T  (A = W2 columns, B = the lane's own dz2[t]); its D element (m, r) is
//                        unit u(4 m + r, g), the lane's own z1 unit, so dZ1 needs no movement.
// The weight gradients sum over the tile's samples: dZ2 and H1 go through LDS (transposed) into
// gW2 = dZ2^T H1 on the matrix cores; gW1, the biases and W3 sum 16 samples per lane.  Each
// tile writes its partial gradient (FP32 sums of 16 samples) and its loss sum; mlp_reduce adds
// the tiles in FP64 in tile order, so the result does not depend on scheduling.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MLP_TILE = 16;  // samples per wavefront

__device__ __forceinline__ int mlp_unit(int t, int g) { return 16 * (t >> 2) + 4 * g + (t & 3); }

__global__ void __launch_bounds__(WAVE) mlp_tile_grad_kernel(const float* __restrict__ theta,
                                                             const float* __restrict__ X,
                                                             const float* __restrict__ y,
                                                             int64_t b0, int B,
                                                             float* __restrict__ partial) {
  __shared__ float sdz2[MLP_TILE][NH + 1];  // dL/dz2 (sample, unit)
  __shared__ float sh1[MLP_TILE][NH + 1];   // h1 = relu(z1)
  __shared__ float sdz1[MLP_TILE][NH + 1];  // dL/dz1
  __shared__ float sh2[MLP_TILE][NH + 1];   // h2 = relu(z2)
  __shared__ float sx[MLP_TILE][NI];
  __shared__ float sdo[MLP_TILE], sr2[MLP_TILE];
  const int l = threadIdx.x, s = l & 15, g = l >> 4;
  const int tile = blockIdx.x;
  const int si = tile * MLP_TILE + s;  // sample within the batch
  const bool valid = si < B;
  const int64_t gs = b0 + (valid ? si : 0);
  const float* W1 = theta + OW1;
  const float* b1 = theta + OB1;
  const float* W2 = theta + OW2;
  const float* b2 = theta + OB2;
  const float* w3 = theta + OW3;
  float x[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) x[c] = valid ? X[4 * gs + c] : 0.0f;
  // layer 1 on the lane's 16 units
  float z1[16], h1[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int u = mlp_unit(t, g);
    float z = b1[u];
#pragma unroll
    for (int c = 0; c < NI; ++c) z = fmaf(W1[u * NI + c], x[c], z);
    z1[t] = z;
    h1[t] = fmaxf(z, 0.0f);
  }
  // Z2^T = W2 H1^T: output tile m holds units 16 m + i (rows) by the 16 samples (columns)
  f32x4 z2v[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 16; ++t)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(W2[(16 * m + s) * NH + mlp_unit(t, g)], h1[t],
                                                 acc, 0, 0, 0);
    z2v[m] = acc;
  }
  // z2 of the lane's sample s at unit 16 m + 4 g + r = u(4 m + r, g); output and residual
  float z2[16], part = 0.0f;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int u = mlp_unit(t, g);
    z2[t] = z2v[t >> 2][t & 3] + b2[u];
    part = fmaf(w3[u], fmaxf(z2[t], 0.0f), part);
  }
  part += __shfl_xor(part, 16, WAVE);
  part += __shfl_xor(part, 32, WAVE);
  const float o = part + theta[OB3];
  const float r = valid ? o - y[gs] : 0.0f;
  const float dout = 2.0f * r / (float)B;  // d(mean of r^2)/do
  // dL/dz2 in the lane's layout (it is also the B operand of the next product)
  float dz2[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int u = mlp_unit(t, g);
    dz2[t] = z2[t] > 0.0f ? dout * w3[u] : 0.0f;
    sdz2[s][u] = dz2[t];
    sh1[s][u] = h1[t];
    sh2[s][u] = fmaxf(z2[t], 0.0f);
  }
  // dH1^T = W2^T dZ2^T: output tile m holds inputs 16 m + i (rows) by the samples
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 16; ++t)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(W2[mlp_unit(t, g) * NH + 16 * m + s], dz2[t],
                                                 acc, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * m + q;  // element q of tile m is unit u(t, g), the lane's z1[t]
      sdz1[s][mlp_unit(t, g)] = z1[t] > 0.0f ? acc[q] : 0.0f;
    }
  }
  if (g == 0) {
#pragma unroll
    for (int c = 0; c < NI; ++c) sx[s][c] = x[c];
    sdo[s] = dout;
    sr2[s] = r * r;
  }
  __syncthreads();
  float* out = partial + (int64_t)tile * (MLP_NPARAMS + 1);
  // gW2 = dZ2^T H1 (64 x 64, summed over the 16 samples): 16 output tiles, k = 4 samples
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int nv = 0; nv < 4; ++nv) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sdz2[4 * k + g][16 * mu + s],
                                                   sh1[4 * k + g][16 * nv + s], acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[OW2 + (16 * mu + 4 * g + q) * NH + 16 * nv + s] = acc[q];
    }
  }
  // lane l = unit u: W1 row, biases and W3 over the 16 samples
  {
    const int u = l;
    float gw1[NI] = {0.0f, 0.0f, 0.0f, 0.0f}, gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f;
#pragma unroll
    for (int q = 0; q < MLP_TILE; ++q) {
      const float d1 = sdz1[q][u];
#pragma unroll
      for (int c = 0; c < NI; ++c) gw1[c] = fmaf(d1, sx[q][c], gw1[c]);
      gb1 += d1;
      gb2 += sdz2[q][u];
      gw3 = fmaf(sdo[q], sh2[q][u], gw3);
    }
#pragma unroll
    for (int c = 0; c < NI; ++c) out[OW1 + u * NI + c] = gw1[c];
    out[OB1 + u] = gb1;
    out[OB2 + u] = gb2;
    out[OW3 + u] = gw3;
  }
  if (l == 0) {
    float gb3 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int q = 0; q < MLP_TILE; ++q) {
      gb3 += sdo[q];
      loss += sr2[q];
    }
    out[OB3] = gb3;
    out[MLP_NPARAMS] = loss;
  }
}

// grad[p] = sum over the tiles of their partial gradients (FP64); p == MLP_NPARAMS gives the
// batch loss (1/B) sum r^2.  A workgroup takes 64 parameters (one per lane); wavefront q sums
// the tiles q, q + 4, q + 8, ... in that order, and the four sums are added in wavefront order,
// so the result is the same on every run.
__global__ void __launch_bounds__(WG) mlp_reduce_kernel(const float* __restrict__ partial,
                                                        int ntiles, int B,
                                                        float* __restrict__ grad) {
  __shared__ double sums[NWAVE][WAVE];
  const int lane = threadIdx.x & (WAVE - 1), q = threadIdx.x / WAVE;
  const int p = blockIdx.x * WAVE + lane;
  double acc = 0.0;
  if (p <= MLP_NPARAMS) {
    const float* col = partial + p;
    int t = q;
    for (; t + 7 * NWAVE < ntiles; t += 8 * NWAVE) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(int64_t)(t + u * NWAVE) * (MLP_NPARAMS + 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; t < ntiles; t += NWAVE) acc += (double)col[(int64_t)t * (MLP_NPARAMS + 1)];
  }
  sums[q][lane] = acc;
  __syncthreads();
  if (q == 0 && p <= MLP_NPARAMS) {
    double a = sums[0][lane];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) a += sums[w][lane];
    grad[p] = (float)(p == MLP_NPARAMS ? a / (double)B : a);
  }
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

// scratch of launch_mlp_grad: one partial gradient (and loss sum) per tile of 16 samples
size_t mlp_cache_floats(int B) {
  return (size_t)((B + MLP_TILE - 1) / MLP_TILE) * (size_t)(MLP_NPARAMS + 1);
}

void launch_mlp_grad(const float* theta, const float* X, const float* y, int64_t b0, int B,
                     float* cache, float* grad, hipStream_t s) {
  const int ntiles = (B + MLP_TILE - 1) / MLP_TILE;
  hipLaunchKernelGGL(mlp_tile_grad_kernel, dim3(ntiles), dim3(WAVE), 0, s, theta, X, y, b0, B,
                     cache);
  HMX_LAUNCHED();
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((MLP_NPARAMS + 1 + WAVE - 1) / WAVE), dim3(WG), 0, s,
                     cache, ntiles, B, grad);
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

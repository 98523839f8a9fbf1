// hmx_mlp.hip -- C ABI of the block-rank MLP: features of an operator's far blocks, inference,
// loss and gradient, training (minibatch Adam), and the process-wide model used by builds with
// HMX_RANK_LEARNED.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hmx_host.h"

using namespace hmx;

namespace hmx {
namespace {
std::mutex g_model_mu;
RankModel g_model;
}  // namespace

RankModel get_rank_model() {
  std::lock_guard<std::mutex> g(g_model_mu);
  return g_model;
}
}  // namespace hmx

namespace {
hmx_status mlp_fail(hmx_status c, const std::string& m) {
  hmx::set_last_error(m);
  return c;
}
}  // namespace

#define MLP_TRY try {
#define MLP_CATCH                                             \
  }                                                           \
  catch (const hmx::Error& e) {                               \
    return mlp_fail(e.code, e.what());                        \
  }                                                           \
  catch (const std::bad_alloc&) {                             \
    return mlp_fail(HMX_ENOMEM, "host allocation failed");    \
  }                                                           \
  catch (const std::exception& e) {                           \
    return mlp_fail(HMX_EINTERNAL, e.what());                 \
  }

extern "C" {

hmx_status hmx_mlp_predict(const float* theta, const float* norm, const float* feat, int64_t n,
                           float* out, void* stream) {
  MLP_TRY
  HMX_REQUIRE(theta && norm && (n == 0 || (feat && out)), HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n >= 0, HMX_EINVAL, "n must be >= 0");
  for (int c = 0; c < 4; ++c)
    HMX_REQUIRE(std::isfinite(norm[4 + c]) && norm[4 + c] > 0, HMX_EINVAL,
                "feature scales must be > 0");
  hipStream_t s = (hipStream_t)stream;
  DevBuf<float> th(MLP_NPARAMS), nm(8);
  HMX_HIP(hipMemcpyAsync(th.p, theta, MLP_NPARAMS * 4, hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemcpyAsync(nm.p, norm, 8 * 4, hipMemcpyHostToDevice, s));
  launch_mlp_predict(th.p, nm.p, feat, n, out, s);
  HMX_HIP(hipStreamSynchronize(s));
  return HMX_OK;
  MLP_CATCH
}

hmx_status hmx_mlp_loss_grad(const float* theta, const float* X, const float* y, int64_t n,
                             float* grad, float* loss, void* stream) {
  MLP_TRY
  HMX_REQUIRE(theta && X && y && grad && loss, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n >= 1 && n <= (int64_t(1) << 24), HMX_EINVAL, "n must be in [1, 2^24]");
  hipStream_t s = (hipStream_t)stream;
  DevBuf<float> th(MLP_NPARAMS), g(MLP_NPARAMS + 1), cache(mlp_cache_floats((int)n));
  HMX_HIP(hipMemcpyAsync(th.p, theta, MLP_NPARAMS * 4, hipMemcpyHostToDevice, s));
  launch_mlp_grad(th.p, X, y, 0, (int)n, cache.p, g.p, s);
  std::vector<float> hg;
  to_host(hg, g.p, MLP_NPARAMS + 1, s);
  std::memcpy(grad, hg.data(), MLP_NPARAMS * 4);
  *loss = hg[MLP_NPARAMS];
  return HMX_OK;
  MLP_CATCH
}

hmx_status hmx_mlp_train(float* theta, const float* X, const float* y, int64_t n, int32_t epochs,
                         int32_t batch, float lr, float* loss_hist, void* stream) {
  MLP_TRY
  HMX_REQUIRE(theta && X && y, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n >= 1 && epochs >= 1 && batch >= 1 && batch <= (1 << 20), HMX_EINVAL,
              "need n >= 1, epochs >= 1, 1 <= batch <= 2^20");
  HMX_REQUIRE(std::isfinite(lr) && lr > 0, HMX_EINVAL, "lr must be > 0");
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)std::min<int64_t>(batch, n);
  const int64_t steps_per_epoch = (n + B - 1) / B;
  DevBuf<float> th(MLP_NPARAMS), g(MLP_NPARAMS + 1), m(MLP_NPARAMS), v(MLP_NPARAMS),
      cache(mlp_cache_floats(B)), losses(steps_per_epoch * epochs);
  HMX_HIP(hipMemcpyAsync(th.p, theta, MLP_NPARAMS * 4, hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemsetAsync(m.p, 0, MLP_NPARAMS * 4, s));
  HMX_HIP(hipMemsetAsync(v.p, 0, MLP_NPARAMS * 4, s));
  int t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t b0 = 0; b0 < n; b0 += B) {
      const int nb = (int)std::min<int64_t>(B, n - b0);
      launch_mlp_grad(th.p, X, y, b0, nb, cache.p, g.p, s);
      HMX_HIP(hipMemcpyAsync(losses.p + t, g.p + MLP_NPARAMS, 4, hipMemcpyDeviceToDevice, s));
      ++t;
      launch_mlp_adam(th.p, g.p, m.p, v.p, t, lr, s);
    }
  }
  std::vector<float> hl, ht;
  to_host(hl, losses.p, (size_t)t, s);
  to_host(ht, th.p, MLP_NPARAMS, s);
  std::memcpy(theta, ht.data(), MLP_NPARAMS * 4);
  if (loss_hist) {
    for (int e = 0; e < epochs; ++e) {
      double a = 0;
      for (int64_t q = 0; q < steps_per_epoch; ++q) a += hl[e * steps_per_epoch + q];
      loss_hist[e] = (float)(a / (double)steps_per_epoch);
    }
  }
  return HMX_OK;
  MLP_CATCH
}

hmx_status hmx_far_features(const hmx_op* op, float* feat) {
  MLP_TRY
  HMX_REQUIRE(op && feat, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no far blocks");
  const int64_t nf = op->n_far;
  if (nf == 0) return HMX_OK;
  DevBuf<float> f(4 * nf);
  launch_mlp_features(op->farL.p, nf, op->nbegin.p, op->nend.p, op->box.p, op->kpt.p, f.p, nullptr);
  std::vector<float> h;
  to_host(h, f.p, 4 * (size_t)nf, nullptr);
  std::memcpy(feat, h.data(), 4 * (size_t)nf * 4);
  return HMX_OK;
  MLP_CATCH
}

hmx_status hmx_set_rank_model(const float* theta, const float* norm, float alpha, float beta) {
  MLP_TRY
  std::lock_guard<std::mutex> g(g_model_mu);
  if (!theta) {
    g_model.set = false;
    return HMX_OK;
  }
  HMX_REQUIRE(norm, HMX_EINVAL, "null norm");
  HMX_REQUIRE(std::isfinite(alpha) && alpha > 0 && std::isfinite(beta) && beta >= 0, HMX_EINVAL,
              "need alpha > 0 and beta >= 0");
  for (int c = 0; c < 4; ++c)
    HMX_REQUIRE(std::isfinite(norm[4 + c]) && norm[4 + c] > 0, HMX_EINVAL,
                "feature scales must be > 0");
  std::memcpy(g_model.theta, theta, sizeof(g_model.theta));
  std::memcpy(g_model.norm, norm, sizeof(g_model.norm));
  g_model.alpha = alpha;
  g_model.beta = beta;
  g_model.set = true;
  return HMX_OK;
  MLP_CATCH
}

}  // extern "C"
